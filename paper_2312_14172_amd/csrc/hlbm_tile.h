// hlbm_tile.h -- tile machinery shared by the gfx950 lattice kernels: pull
// indexing of the structure-of-arrays populations, the tile's particles staged
// in LDS and the per-tile coupling fields (indicator sum S0 and solid-velocity
// sum S1) built by a dense pre-pass over each particle's part of the tile.
//
// Storage: populations as structure of arrays A[i][cell] (x fastest), two
// buffers, pull streaming: the cell x at step t reads f_i(x, t) from
// A[i][x - c_i] (or A[opp i][x] when x - c_i lies past a wall: half-way
// bounce-back).
#pragma once

#include "hlbm_device.h"

namespace hlbm {
// ---------------------------------------------------------------------------
// Pull-index helpers
// ---------------------------------------------------------------------------
struct CellPos {
  int x, y, z;
  bool act;
};

// Source index of f_i(x) in pull storage: A[i][x - c_i], or A[opp i][x] when
// x - c_i lies past a wall.
struct PullIdx {
  int xm, xp, ym, yp, zm, zp;         // wrapped neighbour coordinates (x-1, x+1, ...)
  bool bxm, bxp, bym, byp, bzm, bzp;  // neighbour lies past a wall
  int cell;
};

__device__ inline PullIdx pull_index(const Lattice &L, const CellPos &cp) {
  PullIdx P;
  P.xm = cp.x == 0 ? L.nx - 1 : cp.x - 1;
  P.xp = cp.x == L.nx - 1 ? 0 : cp.x + 1;
  P.ym = cp.y == 0 ? L.ny - 1 : cp.y - 1;
  P.yp = cp.y == L.ny - 1 ? 0 : cp.y + 1;
  P.zm = cp.z == 0 ? L.nz - 1 : cp.z - 1;
  P.zp = cp.z == L.nz - 1 ? 0 : cp.z + 1;
  P.bxm = L.bc[0] && cp.x == 0;
  P.bxp = L.bc[0] && cp.x == L.nx - 1;
  P.bym = L.bc[1] && cp.y == 0;
  P.byp = L.bc[1] && cp.y == L.ny - 1;
  P.bzm = L.bc[2] && cp.z == 0;
  P.bzp = L.bc[2] && cp.z == L.nz - 1;
  P.cell = cp.x + L.nx * (cp.y + L.ny * cp.z);
  return P;
}

template <int I>
__device__ inline long long pull_src(const Lattice &L, const CellPos &cp, const PullIdx &P, int &plane) {
  constexpr int cx = kCX[I], cy = kCY[I], cz = kCZ[I];
  const bool bounce = (cx == 1 && P.bxm) || (cx == -1 && P.bxp) || (cy == 1 && P.bym) ||
                      (cy == -1 && P.byp) || (cz == 1 && P.bzm) || (cz == -1 && P.bzp);
  const int sx = cx == 1 ? P.xm : (cx == -1 ? P.xp : cp.x);
  const int sy = cy == 1 ? P.ym : (cy == -1 ? P.yp : cp.y);
  const int sz = cz == 1 ? P.zm : (cz == -1 ? P.zp : cp.z);
  plane = bounce ? opp(I) : I;
  return bounce ? (long long)P.cell : (long long)sx + (long long)L.nx * (sy + (long long)L.ny * sz);
}

template <class ST, int I = 0>
__device__ inline void pull_all(const Lattice &L, const typename ST::S *__restrict__ A,
                                const CellPos &cp, const PullIdx &P, typename ST::T *g) {
  if constexpr (I < Q) {
    int plane;
    const long long idx = pull_src<I>(L, cp, P, plane);
    g[I] = ST::dec(A[(long long)plane * L.N + idx]);
    pull_all<ST, I + 1>(L, A, cp, P, g);
  }
}

// ---------------------------------------------------------------------------
// Particle -> fluid coupling evaluated inside the lattice kernels
// ---------------------------------------------------------------------------
// Tiles are visited in XCD-contiguous runs (xcd_chunk): the halo rows that
// neighbouring tiles share are read through the same L2.

// A tile's particle, staged in LDS, in the geometry precision G.  Offsets are
// formed as (cell - floor(X)) + (1/2 - frac(X)) so that FP32 keeps the
// fraction exact to its own rounding.
template <typename G>
struct Cand {
  G U[3], W[3];
  G R[9];
  G p0, p1;
  G off[3];      // 1/2 - frac(X)
  G reach2;      // (rc + eps/2)^2: B = 0 beyond
  G inner2;      // (r_in - eps/2)^2 with r_in the inscribed radius: B = 1 within
  G ia2, ib2;    // spheroid: 1 / p0^2, 1 / p1^2
  int Xi[3];     // floor(X)
  int lo[3], hi[3];
  int shape;
  long long tab; // first table entry of a learned particle, -1 for the exact path
  int tsx, tsy;  // coupling-box extents (table strides)
};

template <typename G>
struct TileCands {
  Cand<G> c[MAXC];
  int raw[MAXC];
  int n;
};

// Load the tile's particles into LDS sorted by particle index (so every sum
// over them has a fixed order).  Ends with a barrier.
template <typename G>
__device__ inline void load_candidates(const Lattice &L, const DevParticle *parts, const int *tcnt,
                                       const int *tlist, int tile, TileCands<G> &tc) {
  const int n = min(tcnt[tile], MAXC);
  const int t = threadIdx.x;
  if (t == 0) tc.n = n;
  if (t < n) tc.raw[t] = tlist[tile * MAXC + t];
  __syncthreads();
  if (t < n) {
    const int id = tc.raw[t];
    int rank = 0;
    for (int k = 0; k < n; ++k) rank += (tc.raw[k] < id);
    const DevParticle &p = parts[id];
    Cand<G> &c = tc.c[rank];
    for (int k = 0; k < 3; ++k) {
      c.U[k] = (G)p.U[k];
      c.W[k] = (G)p.W[k];
      const double fl = floor(p.X[k]);
      c.Xi[k] = (int)fl;
      c.off[k] = (G)(0.5 - (p.X[k] - fl));
      c.lo[k] = p.lo[k];
      c.hi[k] = p.hi[k];
    }
    for (int k = 0; k < 9; ++k) c.R[k] = (G)p.R[k];
    c.p0 = (G)p.prm[0];
    c.p1 = (G)p.prm[1];
    const double ro = p.rc + 0.5 * L.eps;
    c.reach2 = (G)(ro * ro);
    // inscribed radius: sphere r, rounded cube h, spheroid min(a, b), mesh
    // (stored by the host) scale x the least distance of its surface from the centre
    const double rin = p.shape == 2 ? fmin(p.prm[0], p.prm[1]) : (p.shape == 3 ? p.prm[2] : p.prm[0]);
    const double ri = rin - 0.5 * L.eps;
    c.inner2 = ri > 0.0 ? (G)(ri * ri) : G(-1);
    c.ia2 = (G)(1.0 / (p.prm[0] * p.prm[0]));
    c.ib2 = (G)(1.0 / (p.prm[1] * p.prm[1]));
    c.shape = p.shape;
    c.tab = (p.learned && L.tables) ? (long long)id * L.table_cap : -1;
    c.tsx = p.hi[0] - p.lo[0] + 1;
    c.tsy = p.hi[1] - p.lo[1] + 1;
  }
  __syncthreads();
}

// v within the (possibly wrapped) cell range [lo, hi] of an axis.
__device__ inline bool in_range(int v, int lo, int hi, int n, int periodic) {
  if (!periodic) return v >= lo && v <= hi;
  int d = v - lo;
  if (d < 0) d += n; else if (d >= n) d -= n;
  if (d < 0) d += n;
  return d <= hi - lo;
}

template <typename G>
__device__ inline G axis_offset(int cell, int xi, G off, int n, int periodic) {
  G d = (G)(cell - xi) + off;
  if (periodic) {
    const G h = G(0.5) * (G)n;
    if (d > h) d -= (G)n;
    else if (d < -h) d += (G)n;
  }
  return d;
}

// Per-tile coupling fields in LDS: for every cell of the tile
//   S0 = sum_p B_p,  S1 = sum_p B_p u_p(x)      (Sec. 3.2; overlap reading:
//   B = min(1, S0), u_s = S1 / S0).
// The tile's particles are processed one after the other in index order; each
// LDS entry is written by one wavefront only (fixed summation order).
template <typename G>
struct TileFields {
  G S0[TZ * TY * TX];
  G S1[3][TZ * TY * TX];
};

// Up to two pieces of [lo, hi] (unwrapped) inside the tile range [t0, t0 + ts)
// of an axis of extent n, as local tile coordinates.
__device__ inline int axis_pieces(int lo, int hi, int t0, int ts, int n, int periodic, int *a, int *b) {
  int cnt = 0;
  const int t1 = min(t0 + ts, n) - 1;
  for (int k = periodic ? -1 : 0; k <= (periodic ? 1 : 0); ++k) {
    const int x0 = max(lo, t0 + k * n), x1 = min(hi, t1 + k * n);
    if (x0 <= x1 && cnt < 2) {
      a[cnt] = x0 - k * n - t0;
      b[cnt] = x1 - k * n - t0;
      ++cnt;
    }
  }
  return cnt;
}

template <typename G>
__device__ inline G cell_indicator(const Lattice &L, const Cand<G> &c, int x, int y, int z, G &d0, G &d1, G &d2,
                                   G he, G eps, G inv_eps) {
  d0 = axis_offset<G>(x, c.Xi[0], c.off[0], L.nx, !L.bc[0]);
  d1 = axis_offset<G>(y, c.Xi[1], c.off[1], L.ny, !L.bc[1]);
  d2 = axis_offset<G>(z, c.Xi[2], c.off[2], L.nz, !L.bc[2]);
  const G r2 = d0 * d0 + d1 * d1 + d2 * d2;
  if (!(r2 < c.reach2)) return G(0);
  if (r2 <= c.inner2) return G(1);  // inside the inscribed sphere shrunk by eps/2
  if (c.tab >= 0) {
    const int lx = box_offset(x, c.lo[0], L.nx, !L.bc[0]);
    const int ly = box_offset(y, c.lo[1], L.ny, !L.bc[1]);
    const int lz = box_offset(z, c.lo[2], L.nz, !L.bc[2]);
    return indicator<G>((G)L.tables[c.tab + lx + c.tsx * (ly + c.tsy * lz)], eps, inv_eps);
  }
  if (c.shape == 0) return indicator<G>(dsqrt(r2) - c.p0, eps, inv_eps);
  const G b0 = c.R[0] * d0 + c.R[3] * d1 + c.R[6] * d2;
  const G b1 = c.R[1] * d0 + c.R[4] * d1 + c.R[7] * d2;
  const G b2 = c.R[2] * d0 + c.R[5] * d1 + c.R[8] * d2;
  return indicator<G>(sdf_for_indicator<G>(c.shape, c.p0, c.p1, c.ia2, c.ib2, b0, b1, b2, he), eps, inv_eps);
}

// Fills tf for tile (tx, ty, tz).  Each wavefront fills the y-row of the tile
// it later collides (cells x = lane, y = wave, all z), so no barrier is
// needed: for each particle in index order, the particle's coupling-box cells
// in that row are spread densely over the wavefront's lanes.  Skips
// everything when the tile has no particles (tf is then not touched).
template <typename G>
__device__ inline void tile_coupling(const Lattice &L, const TileCands<G> &tc, int tx, int ty, int tz,
                                     TileFields<G> &tf) {
  const int nc = tc.n;
  if (nc == 0) return;
  const int w = wave_id(), lane = lane_id();
#pragma unroll
  for (int z = 0; z < TZ; ++z) {
    const int k = lane + TX * (w + TY * z);
    tf.S0[k] = G(0);
    tf.S1[0][k] = tf.S1[1][k] = tf.S1[2][k] = G(0);
  }
  const G he = G(0.5) * (G)L.eps;
  const G eps = (G)L.eps;
  const G inv_eps = (G)(1.0 / L.eps);
  for (int ci = 0; ci < nc; ++ci) {
    const Cand<G> &c = tc.c[ci];
    int ay[2], by[2];
    const int nyp = axis_pieces(c.lo[1], c.hi[1], ty * TY, TY, L.ny, !L.bc[1], ay, by);
    bool row = false;
    for (int py = 0; py < nyp; ++py) row |= (w >= ay[py] && w <= by[py]);
    if (!row) continue;  // uniform per wavefront
    int ax[2], bx[2], az[2], bz[2];
    const int nxp = axis_pieces(c.lo[0], c.hi[0], tx * TX, TX, L.nx, !L.bc[0], ax, bx);
    const int nzp = axis_pieces(c.lo[2], c.hi[2], tz * TZ, TZ, L.nz, !L.bc[2], az, bz);
    for (int pz = 0; pz < nzp; ++pz)
      for (int px = 0; px < nxp; ++px) {
        const int sx = bx[px] - ax[px] + 1, sz = bz[pz] - az[pz] + 1;
        // k -> (x, z) of the piece without integer division: k < 256 and
        // sx <= 64, so floor((k + 1/2) / sx) in FP32 is exact
        const float isx = 1.0f / (float)sx;
        for (int k = lane; k < sx * sz; k += 64) {
          const int kz = (int)(((float)k + 0.5f) * isx);
          const int lx = ax[px] + k - kz * sx, lz = az[pz] + kz;
          G d0, d1, d2;
          const G Bp = cell_indicator<G>(L, c, tx * TX + lx, ty * TY + w, tz * TZ + lz, d0, d1, d2, he, eps,
                                         inv_eps);
          if (Bp > G(0)) {
            const int idx = lx + TX * (w + TY * lz);
            tf.S0[idx] += Bp;
            tf.S1[0][idx] += Bp * (c.U[0] + c.W[1] * d2 - c.W[2] * d1);
            tf.S1[1][idx] += Bp * (c.U[1] + c.W[2] * d0 - c.W[0] * d2);
            tf.S1[2][idx] += Bp * (c.U[2] + c.W[0] * d1 - c.W[1] * d0);
          }
        }
      }
  }
  // the row's LDS writes precede the wavefront's own reads in the cell loop
  __builtin_amdgcn_wave_barrier();
}

}  // namespace hlbm
