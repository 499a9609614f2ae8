// hlbm_kernels.hip -- gfx950 kernels of the HLBM time step.
//
// Storage: populations as structure of arrays A[i][cell] (x fastest), two
// buffers, pull streaming: the cell x at step t reads f_i(x, t) from
// A[i][x - c_i] (or A[opp i][x] when x - c_i lies past a wall: half-way
// bounce-back) and writes its post-collision f*_i(x, t) to B[i][x].
//
// Coupling: particles are binned into 64x4x4 tiles by their reach box; the
// collide kernel evaluates the indicator of the tile's particles at its cells
// (particle -> fluid, EDM), and, after the collision, the momentum exchange
// of the next step from the stored post-collision populations (fluid ->
// particle), reduced per particle with wavefront shuffles in FP64 into one
// partial record per (tile, particle).  A separate pull-form momentum-exchange
// kernel primes the forces whenever the state was set from the host.
#include "hlbm_device.h"
#include "hlbm_internal.h"

namespace hlbm {

__device__ inline int wave_id() { return threadIdx.x >> 6; }
__device__ inline int lane_id() { return threadIdx.x & 63; }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ---------------------------------------------------------------------------
// Particle geometry on the device
// ---------------------------------------------------------------------------
__device__ inline void quat_rot(const double *q, double *R) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

__device__ inline double circumradius(int shape, double p0, double p1) {
  if (shape == 0) return p0;
  if (shape == 1) return 1.7320508075688772 * (p0 - p1) + p1;
  return fmax(p0, p1);
}

// Reach box: cells whose centre lies within `reach` of X along each axis,
// clipped to the domain on wall axes.
__device__ inline void reach_box(const Lattice &L, DevParticle &p) {
  const int n[3] = {L.nx, L.ny, L.nz};
  for (int k = 0; k < 3; ++k) {
    int lo = (int)ceil(p.X[k] - p.reach - 0.5);
    int hi = (int)floor(p.X[k] + p.reach - 0.5);
    if (L.bc[k]) {
      lo = max(lo, 0);
      hi = min(hi, n[k] - 1);
    }
    p.lo[k] = lo;
    p.hi[k] = hi;
  }
}

__device__ inline void derive(const Lattice &L, DevParticle &p) {
  quat_rot(p.q, p.R);
  p.rc = circumradius(p.shape, p.prm[0], p.prm[1]);
  p.reach = p.rc + fmax(0.5 * L.eps, 1.4142135623730951) + 1e-9;
  reach_box(L, p);
}

// Tiles touched by a cell range along one axis (wrapped on periodic axes),
// in increasing cell order; returns the count (<= 16).
__device__ inline int axis_tiles(int lo, int hi, int n, int periodic, int tsize, int *out) {
  int cnt = 0, last = -1;
  for (int c = lo; c <= hi; ++c) {
    int w = c;
    if (periodic) { w %= n; if (w < 0) w += n; }
    if (w < 0 || w >= n) continue;
    const int t = w / tsize;
    if (t != last) {
      bool seen = false;
      for (int k = 0; k < cnt; ++k) seen |= (out[k] == t);
      if (!seen && cnt < 16) out[cnt++] = t;
      last = t;
    }
  }
  return cnt;
}

__global__ void k_prepare(Lattice L, const hlbm_particle *in, DevParticle *out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const hlbm_particle s = in[i];
  DevParticle p;
  for (int k = 0; k < 3; ++k) {
    p.X[k] = s.pos[k]; p.U[k] = s.vel[k]; p.W[k] = s.omega[k];
    p.I[k] = s.inertia[k]; p.prm[k] = s.param[k];
    p.Fh[k] = 0.0; p.Th[k] = 0.0;
  }
  const double nq = sqrt(s.quat[0] * s.quat[0] + s.quat[1] * s.quat[1] + s.quat[2] * s.quat[2] +
                         s.quat[3] * s.quat[3]);
  for (int k = 0; k < 4; ++k) p.q[k] = s.quat[k] / nq;
  p.m = s.mass;
  p.V = s.volume;
  p.shape = s.shape;
  p.flags = s.flags;
  derive(L, p);
  out[i] = p;
}

__global__ void k_fill_int(int *p, int v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// One thread per particle: append the particle to every tile its reach box
// touches.
__global__ void k_bin(Lattice L, const DevParticle *parts, int n, int *tcnt, int *tlist, int *status) {
  const int pid = blockIdx.x * blockDim.x + threadIdx.x;
  if (pid >= n) return;
  const DevParticle &p = parts[pid];
  int tx[16], ty[16], tz[16];
  const int cx = axis_tiles(p.lo[0], p.hi[0], L.nx, !L.bc[0], TX, tx);
  const int cy = axis_tiles(p.lo[1], p.hi[1], L.ny, !L.bc[1], TY, ty);
  const int cz = axis_tiles(p.lo[2], p.hi[2], L.nz, !L.bc[2], TZ, tz);
  for (int c = 0; c < cz; ++c)
    for (int b = 0; b < cy; ++b)
      for (int a = 0; a < cx; ++a) {
        const int t = tx[a] + L.ntx * (ty[b] + L.nty * tz[c]);
        const int slot = atomicAdd(&tcnt[t], 1);
        if (slot < MAXC) tlist[t * MAXC + slot] = pid;
        else atomicOr(status, ST_TILE_OVERFLOW);
      }
}

// One thread per particle: gather the partial momentum-exchange records of the
// tiles the particle was binned to (fixed tile order), add gravity and
// buoyancy, advance the Newton-Euler equations in FP64, refresh the derived
// geometry.
//   U <- U + F/m;  X <- X + U (wrapped on periodic axes);
//   w_b <- w_b + I^-1 (T_b - w_b x I w_b) in the body frame;
//   q <- normalize(q (x) exp(w_b / 2));  w <- R(q) w_b.
__global__ void k_eom(Lattice L, DevParticle *parts, int n, const int *tcnt, const int *tlist,
                      const double *partial, int *status) {
  const int pid = blockIdx.x * blockDim.x + threadIdx.x;
  if (pid >= n) return;
  DevParticle p = parts[pid];
  int tx[16], ty[16], tz[16];
  const int cx = axis_tiles(p.lo[0], p.hi[0], L.nx, !L.bc[0], TX, tx);
  const int cy = axis_tiles(p.lo[1], p.hi[1], L.ny, !L.bc[1], TY, ty);
  const int cz = axis_tiles(p.lo[2], p.hi[2], L.nz, !L.bc[2], TZ, tz);
  double F[3] = {0, 0, 0}, T[3] = {0, 0, 0};
  for (int c = 0; c < cz; ++c)
    for (int b = 0; b < cy; ++b)
      for (int a = 0; a < cx; ++a) {
        const int t = tx[a] + L.ntx * (ty[b] + L.nty * tz[c]);
        const int cnt = min(tcnt[t], MAXC);
        for (int s = 0; s < cnt; ++s) {
          if (tlist[t * MAXC + s] == pid) {
            const double *r = partial + (size_t)(t * MAXC + s) * 6;
            F[0] += r[0]; F[1] += r[1]; F[2] += r[2];
            T[0] += r[3]; T[1] += r[4]; T[2] += r[5];
            break;
          }
        }
      }
  for (int k = 0; k < 3; ++k) { p.Fh[k] = F[k]; p.Th[k] = T[k]; }
  if (p.m > 0.0) {
    const double buoy = p.m - L.rho_f * p.V;
    const int n3[3] = {L.nx, L.ny, L.nz};
    for (int k = 0; k < 3; ++k) {
      p.U[k] += (F[k] + buoy * L.g[k]) / p.m;
      p.X[k] += p.U[k];
      if (!L.bc[k]) {
        if (p.X[k] >= n3[k]) p.X[k] -= n3[k];
        else if (p.X[k] < 0.0) p.X[k] += n3[k];
      } else if (!(p.X[k] >= 0.0 && p.X[k] <= n3[k])) {
        atomicOr(status, ST_WALL_EXIT);
      }
    }
    const double *R = p.R;
    double wb[3], tb[3];
    for (int k = 0; k < 3; ++k) {
      wb[k] = R[0 * 3 + k] * p.W[0] + R[1 * 3 + k] * p.W[1] + R[2 * 3 + k] * p.W[2];
      tb[k] = R[0 * 3 + k] * T[0] + R[1 * 3 + k] * T[1] + R[2 * 3 + k] * T[2];
    }
    const double Iw0 = p.I[0] * wb[0], Iw1 = p.I[1] * wb[1], Iw2 = p.I[2] * wb[2];
    const double g0 = wb[1] * Iw2 - wb[2] * Iw1;
    const double g1 = wb[2] * Iw0 - wb[0] * Iw2;
    const double g2 = wb[0] * Iw1 - wb[1] * Iw0;
    wb[0] += (tb[0] - g0) / p.I[0];
    wb[1] += (tb[1] - g1) / p.I[1];
    wb[2] += (tb[2] - g2) / p.I[2];
    const double ang = sqrt(wb[0] * wb[0] + wb[1] * wb[1] + wb[2] * wb[2]);
    double d0 = 1.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
    if (ang > 0.0) {
      double sn, cs;
      sincos(0.5 * ang, &sn, &cs);
      const double f = sn / ang;
      d0 = cs; d1 = f * wb[0]; d2 = f * wb[1]; d3 = f * wb[2];
    }
    const double *q = p.q;
    double qn[4] = {q[0] * d0 - q[1] * d1 - q[2] * d2 - q[3] * d3,
                    q[0] * d1 + q[1] * d0 + q[2] * d3 - q[3] * d2,
                    q[0] * d2 - q[1] * d3 + q[2] * d0 + q[3] * d1,
                    q[0] * d3 + q[1] * d2 - q[2] * d1 + q[3] * d0};
    const double nq = sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
    for (int k = 0; k < 4; ++k) p.q[k] = qn[k] / nq;
    quat_rot(p.q, p.R);
    for (int k = 0; k < 3; ++k) p.W[k] = p.R[k * 3 + 0] * wb[0] + p.R[k * 3 + 1] * wb[1] + p.R[k * 3 + 2] * wb[2];
    if (!(p.X[0] == p.X[0] && p.X[1] == p.X[1] && p.X[2] == p.X[2])) atomicOr(status, ST_UNSTABLE);
    reach_box(L, p);
  }
  parts[pid] = p;
}

// ---------------------------------------------------------------------------
// Tile set-up shared by the lattice kernels
// ---------------------------------------------------------------------------
struct TileCands {
  Cand c[MAXC];
  int raw[MAXC];
  int n;
};

// Load the tile's particles into LDS sorted by particle index (so every sum
// over them has a fixed order).  Ends with a barrier.
__device__ inline void load_candidates(const Lattice &L, const DevParticle *parts, const int *tcnt,
                                       const int *tlist, int tile, TileCands &tc) {
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
    Cand &c = tc.c[rank];
    for (int k = 0; k < 3; ++k) { c.X[k] = p.X[k]; c.U[k] = p.U[k]; c.W[k] = p.W[k]; }
    for (int k = 0; k < 9; ++k) c.R[k] = p.R[k];
    c.p0 = p.prm[0];
    c.p1 = p.prm[1];
    c.reach2 = p.reach * p.reach;
    c.shape = p.shape;
    c.slot = t;
  }
  __syncthreads();
}

struct CellPos {
  int x, y, z;
  bool act;
};

__device__ inline void cell_offset(const Lattice &L, const Cand &c, const CellPos &cp, double *d) {
  d[0] = min_image((cp.x + 0.5) - c.X[0], L.nx, !L.bc[0]);
  d[1] = min_image((cp.y + 0.5) - c.X[1], L.ny, !L.bc[1]);
  d[2] = min_image((cp.z + 0.5) - c.X[2], L.nz, !L.bc[2]);
}

__device__ inline void to_body(const Cand &c, const double *d, double *b) {
  b[0] = c.R[0] * d[0] + c.R[3] * d[1] + c.R[6] * d[2];
  b[1] = c.R[1] * d[0] + c.R[4] * d[1] + c.R[7] * d[2];
  b[2] = c.R[2] * d[0] + c.R[5] * d[1] + c.R[8] * d[2];
}

// Is the neighbour x + c in the domain (walls only exclude)?
__device__ inline bool nb_valid(const Lattice &L, const CellPos &cp, int cx, int cy, int cz) {
  bool ok = true;
  if (L.bc[0]) { const int v = cp.x + cx; ok &= (v >= 0 && v < L.nx); }
  if (L.bc[1]) { const int v = cp.y + cy; ok &= (v >= 0 && v < L.ny); }
  if (L.bc[2]) { const int v = cp.z + cz; ok &= (v >= 0 && v < L.nz); }
  return ok;
}

// S0 = sum_p B_p and S1 = sum_p B_p u_p(x) over the tile's particles at one
// cell (Sec. 3.2; overlap rule B = min(1, S0), u_s = S1 / S0).
__device__ inline void coupling_at(const Lattice &L, const TileCands &tc, const CellPos &cp,
                                   double &S0, double *S1) {
  S0 = 0.0;
  S1[0] = S1[1] = S1[2] = 0.0;
  const double he = 0.5 * L.eps;
  for (int ci = 0; ci < tc.n; ++ci) {
    const Cand &c = tc.c[ci];
    double d[3];
    cell_offset(L, c, cp, d);
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const bool near = cp.act && r2 <= c.reach2;
    if (__ballot(near) == 0) continue;
    if (near) {
      double ds;
      if (c.shape == 0) {
        ds = sqrt(r2) - c.p0;
      } else {
        double b[3];
        to_body(c, d, b);
        ds = sdf_for_indicator(c.shape, c.p0, c.p1, b[0], b[1], b[2], he);
      }
      if (ds < he) {
        const double Bp = indicator(ds, L.eps);
        S0 += Bp;
        S1[0] += Bp * (c.U[0] + c.W[1] * d[2] - c.W[2] * d[1]);
        S1[1] += Bp * (c.U[1] + c.W[2] * d[0] - c.W[0] * d[2]);
        S1[2] += Bp * (c.U[2] + c.W[0] * d[1] - c.W[1] * d[0]);
      }
    }
  }
}

// Source index of f_i(x) in pull storage: A[i][x - c_i], or A[opp i][x] when
// x - c_i lies past a wall.
struct PullIdx {
  int xm, xp, ym, yp, zm, zp;  // wrapped neighbour coordinates (x-1, x+1, ...)
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

template <class ST, int I>
__device__ inline void pull_one(const Lattice &L, const typename ST::S *__restrict__ A,
                                const CellPos &cp, const PullIdx &P, typename ST::T *g) {
  int plane;
  const long long idx = pull_src<I>(L, cp, P, plane);
  g[I] = ST::dec(A[(long long)plane * L.N + idx], I);
}

template <class ST, int I = 0>
__device__ inline void pull_all(const Lattice &L, const typename ST::S *__restrict__ A,
                                const CellPos &cp, const PullIdx &P, typename ST::T *g) {
  if constexpr (I < Q) {
    pull_one<ST, I>(L, A, cp, P, g);
    pull_all<ST, I + 1>(L, A, cp, P, g);
  }
}

// Momentum-exchange contributions of one cell for one particle, with the
// populations at time t given per direction through `fin` (f_i(x + c_i, t))
// and `fout` (f_opp(i)(x, t)) when the cell is inside (pull form), or with the
// cell's stored post-collision populations `fs` (push form, see k_collide).
__device__ inline void cross_add(const double *a, const double *b, double *o) {
  o[0] += a[1] * b[2] - a[2] * b[1];
  o[1] += a[2] * b[0] - a[0] * b[2];
  o[2] += a[0] * b[1] - a[1] * b[0];
}

template <class ST>
__device__ inline void reduce_to_lds(double *F, double *T, double (*acc)[MAXC][6], int ci) {
  double v[6] = {F[0], F[1], F[2], T[0], T[1], T[2]};
#pragma unroll
  for (int k = 0; k < 6; ++k) v[k] = wave_sum(v[k]);
  if (lane_id() == 0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[wave_id()][ci][k] += v[k];
  }
}

// Fused collide + stream with the EDM source and the momentum exchange of
// the next step.  One workgroup per tile.
//   rho = 1 + sum g_i,  u = sum c_i g_i / rho                (Sec. 3.1)
//   du = B (u_s - u) + (1 - B) a_f                           (Sec. 3.2)
//   g*_i = (1 - 1/tau)(g_i - geq_i(rho, u)) + geq_i(rho, u + du)
// which is f_i - (f_i - feq_i)/tau + feq_i(u + du) - feq_i(u) written for
// deviations g = f - w, geq = feq - w.
//
// Momentum exchange of step t+1 (uses f(t+1), i.e. this step's stored
// post-collision values, and the particles already advanced to t+1):
//   F_h(x_b) = sum_i (c_i - u_p(x_b)) f_i(x_b + c_i) + (c_i + u_p(x_b)) f_opp(i)(x_b)
// with f_i(x_b + c_i, t+1) = f*_i(x_b, t) (own cell) and
// f_opp(i)(x_b, t+1) = f*_opp(i)(x_b + c_i, t) (the neighbour's own value).
// Each cell therefore adds, for every particle p:
//   if x in x_b(p):            -sum_i (c_i - u_p(x)) f*_i(x)           (lever x)
//   for each j, x + c_j in x_b: -(u_p(x + c_j) - c_j) f*_j(x)          (lever x + c_j)
// (directions whose neighbour lies past a wall are skipped), which is the
// negative of the printed F_h: the force on the particle.
template <class ST>
__global__ __launch_bounds__(256) void k_collide(Lattice L, const typename ST::S *__restrict__ A,
                                                 typename ST::S *__restrict__ Bo,
                                                 const DevParticle *__restrict__ parts,
                                                 const int *__restrict__ tcnt,
                                                 const int *__restrict__ tlist,
                                                 double *__restrict__ partial, int *status) {
  using T = typename ST::T;
  using S = typename ST::S;
  __shared__ TileCands tc;
  __shared__ double acc[4][MAXC][6];
  const int tile = blockIdx.x;
  const int tx = tile % L.ntx;
  const int ty = (tile / L.ntx) % L.nty;
  const int tz = tile / (L.ntx * L.nty);
  load_candidates(L, parts, tcnt, tlist, tile, tc);
  const int nc = tc.n;
  for (int k = threadIdx.x; k < 4 * MAXC * 6; k += blockDim.x) (&acc[0][0][0])[k] = 0.0;
  __syncthreads();

  const T omega = (T)L.omega;
  const T afx = (T)L.af[0], afy = (T)L.af[1], afz = (T)L.af[2];
  const bool has_af = (L.af[0] != 0.0) || (L.af[1] != 0.0) || (L.af[2] != 0.0);

  for (int zz = 0; zz < TZ; ++zz) {
    CellPos cp;
    cp.x = tx * TX + lane_id();
    cp.y = ty * TY + wave_id();
    cp.z = tz * TZ + zz;
    if (cp.z >= L.nz) break;
    cp.act = cp.x < L.nx && cp.y < L.ny;

    T g[Q];
    T gs[Q];
    long long cell = 0;
    if (cp.act) {
      const PullIdx P = pull_index(L, cp);
      cell = P.cell;
      pull_all<ST>(L, A, cp, P, g);
    } else {
#pragma unroll
      for (int i = 0; i < Q; ++i) g[i] = (T)0;
    }
    // moments of the deviations
    T rho1 = (T)0, jx = (T)0, jy = (T)0, jz = (T)0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      rho1 += g[i];
      if (kCX[i]) jx += kCX[i] * g[i];
      if (kCY[i]) jy += kCY[i] * g[i];
      if (kCZ[i]) jz += kCZ[i] * g[i];
    }
    const T rho = (T)1 + rho1;
    const T inv = (T)1 / rho;
    const T ux = jx * inv, uy = jy * inv, uz = jz * inv;

    // particle -> fluid coupling at this cell
    double S0 = 0.0, S1[3] = {0.0, 0.0, 0.0};
    if (nc > 0) coupling_at(L, tc, cp, S0, S1);
    const bool coupled = has_af || S0 > 0.0;
    T du0 = (T)0, du1 = (T)0, du2 = (T)0;
    if (S0 > 0.0) {
      const double Bc = S0 < 1.0 ? S0 : 1.0;
      const T Bt = (T)Bc;
      const T usx = (T)(S1[0] / S0), usy = (T)(S1[1] / S0), usz = (T)(S1[2] / S0);
      du0 = Bt * (usx - ux) + ((T)1 - Bt) * afx;
      du1 = Bt * (usy - uy) + ((T)1 - Bt) * afy;
      du2 = Bt * (usz - uz) + ((T)1 - Bt) * afz;
    } else {
      du0 = afx; du1 = afy; du2 = afz;
    }

    const T usq = ux * ux + uy * uy + uz * uz;
    if (cp.act && !(rho > (T)0 && usq < (T)0.09)) atomicOr(status, ST_UNSTABLE);
    const T vx = ux + du0, vy = uy + du1, vz = uz + du2;
    const T vsq = vx * vx + vy * vy + vz * vz;
    const T one_m_omega = (T)1 - omega;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const T w = (T)wgt(i);
      const T cu = (T)kCX[i] * ux + (T)kCY[i] * uy + (T)kCZ[i] * uz;
      const T geq = w * (rho1 + rho * ((T)3 * cu + (T)4.5 * cu * cu - (T)1.5 * usq));
      if (coupled) {
        const T cv = (T)kCX[i] * vx + (T)kCY[i] * vy + (T)kCZ[i] * vz;
        const T geq2 = w * (rho1 + rho * ((T)3 * cv + (T)4.5 * cv * cv - (T)1.5 * vsq));
        gs[i] = one_m_omega * (g[i] - geq) + geq2;
      } else {
        gs[i] = g[i] - omega * (g[i] - geq);
      }
    }
    if (cp.act) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const S s = ST::enc(gs[i], i);
        Bo[(long long)i * L.N + cell] = s;
        gs[i] = ST::dec(s, i);  // the value the next step will read
      }
    }

    // fluid -> particle: momentum exchange of the next step
    for (int ci = 0; ci < nc; ++ci) {
      const Cand &c = tc.c[ci];
      double d[3];
      cell_offset(L, c, cp, d);
      const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      const bool near = cp.act && r2 <= c.reach2;
      if (__ballot(near) == 0) continue;
      double F[3] = {0, 0, 0}, Tq[3] = {0, 0, 0};
      if (near) {
        double b[3] = {d[0], d[1], d[2]};
        if (c.shape != 0) to_body(c, d, b);
        const double upx = c.U[0] + c.W[1] * d[2] - c.W[2] * d[1];
        const double upy = c.U[1] + c.W[2] * d[0] - c.W[0] * d[2];
        const double upz = c.U[2] + c.W[0] * d[1] - c.W[1] * d[0];
        if (inside_body(c.shape, c.p0, c.p1, b[0], b[1], b[2])) {
          double h[3] = {0, 0, 0};
#pragma unroll
          for (int i = 1; i < Q; ++i) {
            if (!nb_valid(L, cp, kCX[i], kCY[i], kCZ[i])) continue;
            const double f = (double)gs[i] + wgt(i);
            h[0] += (kCX[i] - upx) * f;
            h[1] += (kCY[i] - upy) * f;
            h[2] += (kCZ[i] - upz) * f;
          }
          F[0] -= h[0]; F[1] -= h[1]; F[2] -= h[2];
          const double mh[3] = {-h[0], -h[1], -h[2]};
          cross_add(d, mh, Tq);
        }
#pragma unroll
        for (int j = 1; j < Q; ++j) {
          if (!nb_valid(L, cp, kCX[j], kCY[j], kCZ[j])) continue;
          double bj[3];
          if (c.shape == 0) {
            bj[0] = d[0] + kCX[j]; bj[1] = d[1] + kCY[j]; bj[2] = d[2] + kCZ[j];
          } else {
            bj[0] = b[0] + c.R[0] * kCX[j] + c.R[3] * kCY[j] + c.R[6] * kCZ[j];
            bj[1] = b[1] + c.R[1] * kCX[j] + c.R[4] * kCY[j] + c.R[7] * kCZ[j];
            bj[2] = b[2] + c.R[2] * kCX[j] + c.R[5] * kCY[j] + c.R[8] * kCZ[j];
          }
          if (!inside_body(c.shape, c.p0, c.p1, bj[0], bj[1], bj[2])) continue;
          const double dj[3] = {d[0] + kCX[j], d[1] + kCY[j], d[2] + kCZ[j]};
          const double vjx = upx + c.W[1] * kCZ[j] - c.W[2] * kCY[j];
          const double vjy = upy + c.W[2] * kCX[j] - c.W[0] * kCZ[j];
          const double vjz = upz + c.W[0] * kCY[j] - c.W[1] * kCX[j];
          const double f = (double)gs[j] + wgt(j);
          const double h[3] = {(vjx - kCX[j]) * f, (vjy - kCY[j]) * f, (vjz - kCZ[j]) * f};
          F[0] -= h[0]; F[1] -= h[1]; F[2] -= h[2];
          const double mh[3] = {-h[0], -h[1], -h[2]};
          cross_add(dj, mh, Tq);
        }
      }
      reduce_to_lds<ST>(F, Tq, acc, ci);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nc * 6; k += blockDim.x) {
    const int ci = k / 6, comp = k % 6;
    const double v = acc[0][ci][comp] + acc[1][ci][comp] + acc[2][ci][comp] + acc[3][ci][comp];
    partial[(size_t)(tile * MAXC + tc.c[ci].slot) * 6 + comp] = v;
  }
}

// Pull-form momentum exchange from the stored state (used when the state was
// set from the host).  For x in x_b and every direction i with x + c_i in the
// domain: f_i(x + c_i, t) = A[i][x] and f_opp(i)(x, t) = A[opp i][x + c_i].
template <class ST>
__global__ __launch_bounds__(256) void k_mea_pull(Lattice L, const typename ST::S *__restrict__ A,
                                                  const DevParticle *__restrict__ parts,
                                                  const int *__restrict__ tcnt,
                                                  const int *__restrict__ tlist,
                                                  double *__restrict__ partial) {
  __shared__ TileCands tc;
  __shared__ double acc[4][MAXC][6];
  const int tile = blockIdx.x;
  const int tx = tile % L.ntx;
  const int ty = (tile / L.ntx) % L.nty;
  const int tz = tile / (L.ntx * L.nty);
  load_candidates(L, parts, tcnt, tlist, tile, tc);
  const int nc = tc.n;
  if (nc == 0) return;
  for (int k = threadIdx.x; k < 4 * MAXC * 6; k += blockDim.x) (&acc[0][0][0])[k] = 0.0;
  __syncthreads();
  for (int zz = 0; zz < TZ; ++zz) {
    CellPos cp;
    cp.x = tx * TX + lane_id();
    cp.y = ty * TY + wave_id();
    cp.z = tz * TZ + zz;
    if (cp.z >= L.nz) break;
    cp.act = cp.x < L.nx && cp.y < L.ny;
    const long long cell = cp.act ? cp.x + (long long)L.nx * (cp.y + (long long)L.ny * cp.z) : 0;
    for (int ci = 0; ci < nc; ++ci) {
      const Cand &c = tc.c[ci];
      double d[3];
      cell_offset(L, c, cp, d);
      const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      bool in = false;
      if (cp.act && r2 <= c.reach2) {
        double b[3] = {d[0], d[1], d[2]};
        if (c.shape != 0) to_body(c, d, b);
        in = inside_body(c.shape, c.p0, c.p1, b[0], b[1], b[2]);
      }
      if (__ballot(in) == 0) continue;
      double F[3] = {0, 0, 0}, Tq[3] = {0, 0, 0};
      if (in) {
        const double upx = c.U[0] + c.W[1] * d[2] - c.W[2] * d[1];
        const double upy = c.U[1] + c.W[2] * d[0] - c.W[0] * d[2];
        const double upz = c.U[2] + c.W[0] * d[1] - c.W[1] * d[0];
        double h[3] = {0, 0, 0};
#pragma unroll
        for (int i = 1; i < Q; ++i) {
          if (!nb_valid(L, cp, kCX[i], kCY[i], kCZ[i])) continue;
          int nx_ = cp.x + kCX[i], ny_ = cp.y + kCY[i], nz_ = cp.z + kCZ[i];
          if (nx_ < 0) nx_ += L.nx; else if (nx_ >= L.nx) nx_ -= L.nx;
          if (ny_ < 0) ny_ += L.ny; else if (ny_ >= L.ny) ny_ -= L.ny;
          if (nz_ < 0) nz_ += L.nz; else if (nz_ >= L.nz) nz_ -= L.nz;
          const long long nb = nx_ + (long long)L.nx * (ny_ + (long long)L.ny * nz_);
          const double fin = (double)ST::dec(A[(long long)i * L.N + cell], i) + wgt(i);
          const double fout = (double)ST::dec(A[(long long)opp(i) * L.N + nb], opp(i)) + wgt(i);
          h[0] += (kCX[i] - upx) * fin + (kCX[i] + upx) * fout;
          h[1] += (kCY[i] - upy) * fin + (kCY[i] + upy) * fout;
          h[2] += (kCZ[i] - upz) * fin + (kCZ[i] + upz) * fout;
        }
        F[0] = -h[0]; F[1] = -h[1]; F[2] = -h[2];
        const double mh[3] = {-h[0], -h[1], -h[2]};
        cross_add(d, mh, Tq);
      }
      reduce_to_lds<ST>(F, Tq, acc, ci);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nc * 6; k += blockDim.x) {
    const int ci = k / 6, comp = k % 6;
    const double v = acc[0][ci][comp] + acc[1][ci][comp] + acc[2][ci][comp] + acc[3][ci][comp];
    partial[(size_t)(tile * MAXC + tc.c[ci].slot) * 6 + comp] = v;
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
  double dev[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double cu = kCX[i] * u0 + kCY[i] * u1 + kCZ[i] * u2;
    dev[i] = wgt(i) * ((r - 1.0) + r * (3.0 * cu + 4.5 * cu * cu - 1.5 * usq));
  }
#define HLBM_SET_ONE(I)                                                   \
  {                                                                       \
    int plane;                                                            \
    const long long idx = pull_src<I>(L, cp, P, plane);                   \
    A[(long long)plane * L.N + idx] = ST::enc((typename ST::T)dev[I], I); \
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
  __shared__ TileCands tc;
  const int tile = blockIdx.x;
  const int tx = tile % L.ntx;
  const int ty = (tile / L.ntx) % L.nty;
  const int tz = tile / (L.ntx * L.nty);
  load_candidates(L, parts, tcnt, tlist, tile, tc);
  for (int zz = 0; zz < TZ; ++zz) {
    CellPos cp;
    cp.x = tx * TX + lane_id();
    cp.y = ty * TY + wave_id();
    cp.z = tz * TZ + zz;
    if (cp.z >= L.nz) break;
    cp.act = cp.x < L.nx && cp.y < L.ny;
    T g[Q];
    long long cell = 0;
    if (cp.act) {
      const PullIdx P = pull_index(L, cp);
      cell = P.cell;
      pull_all<ST>(L, A, cp, P, g);
    }
    double S0 = 0.0, S1[3] = {0, 0, 0};
    if (tc.n > 0) coupling_at(L, tc, cp, S0, S1);
    if (!cp.act) continue;
    double rho1 = 0, j[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double gi = (double)g[i];
      rho1 += gi;
      j[0] += kCX[i] * gi; j[1] += kCY[i] * gi; j[2] += kCZ[i] * gi;
    }
    const double rho = 1.0 + rho1;
    const double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    const double Bc = S0 < 1.0 ? S0 : 1.0;
    double up[3];
    for (int k = 0; k < 3; ++k) {
      const double us = S0 > 0.0 ? S1[k] / S0 : 0.0;
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

hipError_t launch_prepare(const Lattice &L, const hlbm_particle *in, DevParticle *out, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_prepare, dim3(blocks_for(n, 128)), dim3(128), 0, s, L, in, out, n);
  return hipGetLastError();
}

hipError_t launch_fill_int(int *p, int v, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_int, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_bin(const Lattice &L, const DevParticle *parts, int n, int *tcnt, int *tlist, int *status,
                      hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bin, dim3(blocks_for(n, 64)), dim3(64), 0, s, L, parts, n, tcnt, tlist, status);
  return hipGetLastError();
}

hipError_t launch_eom(const Lattice &L, DevParticle *parts, int n, const int *tcnt, const int *tlist,
                      const double *partial, int *status, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_eom, dim3(blocks_for(n, 64)), dim3(64), 0, s, L, parts, n, tcnt, tlist, partial,
                     status);
  return hipGetLastError();
}

hipError_t launch_collide(int prec, const Lattice &L, const void *A, void *B, const DevParticle *parts,
                          const int *tcnt, const int *tlist, double *partial, int *status, hipStream_t s) {
  HLBM_DISPATCH(prec, hipLaunchKernelGGL(k_collide<ST>, dim3(L.ntiles), dim3(256), 0, s, L,
                                         (const typename ST::S *)A, (typename ST::S *)B, parts, tcnt,
                                         tlist, partial, status));
  return hipGetLastError();
}

hipError_t launch_mea_pull(int prec, const Lattice &L, const void *A, const DevParticle *parts,
                           const int *tcnt, const int *tlist, double *partial, hipStream_t s) {
  HLBM_DISPATCH(prec, hipLaunchKernelGGL(k_mea_pull<ST>, dim3(L.ntiles), dim3(256), 0, s, L,
                                         (const typename ST::S *)A, parts, tcnt, tlist, partial));
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
