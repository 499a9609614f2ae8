// hlbm_lattice.hip -- gfx950 lattice kernels of the HLBM time step.
//
// Storage: populations as structure of arrays A[i][cell] (x fastest), two
// buffers, pull streaming: the cell x at step t reads f_i(x, t) from
// A[i][x - c_i] (or A[opp i][x] when x - c_i lies past a wall: half-way
// bounce-back) and writes its post-collision f*_i(x, t) to B[i][x].
//
//   k_collide   one workgroup per tile of 64 x 4 x 4 cells: the tile's
//               particles staged in LDS, the indicator and solid velocity of
//               the tile's cells accumulated in LDS by a dense pre-pass over
//               each particle's part of the tile, then per cell: pull,
//               moments, exact-difference source, BGK, store;
//   k_set_fields / k_fields   equilibrium initialisation and observables.
#include "hlbm_device.h"
#include "hlbm_internal.h"

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

template <class ST>
__global__ __launch_bounds__(256) void k_collide(Lattice L, const typename ST::S *__restrict__ A,
                                                 typename ST::S *__restrict__ Bo,
                                                 const DevParticle *__restrict__ parts,
                                                 const int *__restrict__ tcnt,
                                                 const int *__restrict__ tlist, int *tcnt_clear,
                                                 int *status) {
  using T = typename ST::T;
  using G = typename ST::G;
  __shared__ TileCands<G> tc;
  __shared__ TileFields<G> tf;
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
    if (cp.act && !(rho > (T)0 && usq < (T)0.09)) atomicOr(status, ST_UNSTABLE);
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
  }
}

// f_i(x) = feq_i(rho(x), u(x)) written to its pull-storage slot.
template <class ST>
__global__ void k_set_fields(Lattice L, typename ST::S *__restrict__ A, const double *__restrict__ rho,
                             const double *__restrict__ u) {
  const long long cell = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (cell >= L.N) return;
  CellPos cp;
  cp.x = (int)(cell % L.nx);
  cp.y = (int)((cell / L.nx) % L.ny);
  cp.z = (int)(cell / ((long long)L.nx * L.ny));
  cp.act = true;
  const PullIdx P = pull_index(L, cp);
  const double r = rho ? rho[cell] : 1.0;
  const double u0 = u ? u[cell] : 0.0, u1 = u ? u[L.N + cell] : 0.0, u2 = u ? u[2 * L.N + cell] : 0.0;
  const double usq = u0 * u0 + u1 * u1 + u2 * u2;
  double dev[Q];  // K (feq_i - w_i) / w_i
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double cu = kCX[i] * u0 + kCY[i] * u1 + kCZ[i] * u2;
    dev[i] = (double)ST::K() * ((r - 1.0) + r * (3.0 * cu + 4.5 * cu * cu - 1.5 * usq));
  }
#define HLBM_SET_ONE(I)                                                   \
  {                                                                       \
    int plane;                                                            \
    const long long idx = pull_src<I>(L, cp, P, plane);                   \
    A[(long long)plane * L.N + idx] = ST::enc((typename ST::T)dev[I]);    \
  }
  HLBM_SET_ONE(0) HLBM_SET_ONE(1) HLBM_SET_ONE(2) HLBM_SET_ONE(3) HLBM_SET_ONE(4)
  HLBM_SET_ONE(5) HLBM_SET_ONE(6) HLBM_SET_ONE(7) HLBM_SET_ONE(8) HLBM_SET_ONE(9)
  HLBM_SET_ONE(10) HLBM_SET_ONE(11) HLBM_SET_ONE(12) HLBM_SET_ONE(13) HLBM_SET_ONE(14)
  HLBM_SET_ONE(15) HLBM_SET_ONE(16) HLBM_SET_ONE(17) HLBM_SET_ONE(18)
#undef HLBM_SET_ONE
}

// Observables of the current state: rho, bare u, u_phys = u + du/2 and B,
// written as FP64 planes (order rho, u, u_phys, B; only the selected ones).
template <class ST>
__global__ __launch_bounds__(256) void k_fields(Lattice L, const typename ST::S *__restrict__ A,
                                                const DevParticle *__restrict__ parts,
                                                const int *__restrict__ tcnt,
                                                const int *__restrict__ tlist, unsigned mask,
                                                double *__restrict__ out) {
  using T = typename ST::T;
  using G = typename ST::G;
  __shared__ TileCands<G> tc;
  __shared__ TileFields<G> tf;
  const int tile = xcd_chunk(blockIdx.x, L.ntiles);
  const int tx = tile % L.ntx;
  const int ty = (tile / L.ntx) % L.nty;
  const int tz = tile / (L.ntx * L.nty);
  load_candidates<G>(L, parts, tcnt, tlist, tile, tc);
  tile_coupling<G>(L, tc, tx, ty, tz, tf);
  for (int zz = 0; zz < TZ; ++zz) {
    CellPos cp;
    cp.x = tx * TX + lane_id();
    cp.y = ty * TY + wave_id();
    cp.z = tz * TZ + zz;
    if (cp.z >= L.nz || cp.y >= L.ny) break;
    cp.act = cp.x < L.nx;
    if (!cp.act) continue;
    T g[Q];
    const PullIdx P = pull_index(L, cp);
    const long long cell = P.cell;
    pull_all<ST>(L, A, cp, P, g);
    G S0 = G(0), S1[3] = {G(0), G(0), G(0)};
    if (tc.n > 0) {
      const int idx = lane_id() + TX * (wave_id() + TY * zz);
      S0 = tf.S0[idx];
      S1[0] = tf.S1[0][idx]; S1[1] = tf.S1[1][idx]; S1[2] = tf.S1[2][idx];
    }
    double rho1 = 0, j[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double gi = wgt(i) * (double)g[i] / (double)ST::K();  // f_i - w_i
      rho1 += gi;
      j[0] += kCX[i] * gi; j[1] += kCY[i] * gi; j[2] += kCZ[i] * gi;
    }
    const double rho = 1.0 + rho1;
    const double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    const double s0 = (double)S0;
    const double Bc = s0 < 1.0 ? s0 : 1.0;
    double up[3];
    for (int k = 0; k < 3; ++k) {
      const double us = s0 > 0.0 ? (double)S1[k] / s0 : 0.0;
      const double du = Bc * (us - u[k]) + (1.0 - Bc) * L.af[k];
      up[k] = u[k] + 0.5 * du;
    }
    long long plane = 0;
    if (mask & 1u) { out[plane * L.N + cell] = rho; plane += 1; }
    if (mask & 2u) { for (int k = 0; k < 3; ++k) out[(plane + k) * L.N + cell] = u[k]; plane += 3; }
    if (mask & 4u) { for (int k = 0; k < 3; ++k) out[(plane + k) * L.N + cell] = up[k]; plane += 3; }
    if (mask & 8u) { out[plane * L.N + cell] = Bc; }
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
                          const int *tcnt, const int *tlist, int *tcnt_clear, int *status, hipStream_t s) {
  HLBM_DISPATCH(prec, hipLaunchKernelGGL(k_collide<ST>, dim3(L.ntiles), dim3(256), 0, s, L,
                                         (const typename ST::S *)A, (typename ST::S *)B, parts, tcnt,
                                         tlist, tcnt_clear, status));
  return hipGetLastError();
}

hipError_t launch_set_fields(int prec, const Lattice &L, void *A, const double *rho, const double *u,
                             hipStream_t s) {
  HLBM_DISPATCH(prec, hipLaunchKernelGGL(k_set_fields<ST>, dim3(blocks_for(L.N, 256)), dim3(256), 0, s,
                                         L, (typename ST::S *)A, rho, u));
  return hipGetLastError();
}

hipError_t launch_fields(int prec, const Lattice &L, const void *A, const DevParticle *parts,
                         const int *tcnt, const int *tlist, unsigned mask, double *out, hipStream_t s) {
  HLBM_DISPATCH(prec, hipLaunchKernelGGL(k_fields<ST>, dim3(L.ntiles), dim3(256), 0, s, L,
                                         (const typename ST::S *)A, parts, tcnt, tlist, mask, out));
  return hipGetLastError();
}

}  // namespace hlbm
