// hlbm_particles.hip -- gfx950 kernels of the particle side of the HLBM time
// step: particle set-up, binning into tile lists, momentum exchange and the
// FP64 equations of motion.
//
// Per step (Sec. 4.2, time-step order of Algorithm 1), before the lattice kernel:
//   k_mea      one workgroup per (particle, slab of z-layers of its bounding
//              box): momentum exchange over the slab's inside cells (compacted
//              in LDS), read in pull form from the stored state, FP64 shuffle
//              reduction to a slab record;
//   k_eom_bin  one workgroup per particle: the slab records summed in a fixed
//              order, gravity and buoyancy, Newton-Euler and quaternion update
//              in FP64, then the particle appended to the tile lists of its new
//              coupling box (tiles of 64 x 4 x 4 cells);
//   k_contact_pairs, or k_cgrid_* and k_contact, then k_contact_shapes
//              (only with contact set): the contact pair search (all pairs,
//              or a grid of the centres from 4096 particles on) and the
//              repulsion forces, launched between the two and added to the
//              force by k_eom_bin.
#include <climits>

#include "hlbm_device.h"
#include "hlbm_internal.h"

namespace hlbm {



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
  if (shape == 3) return p1;  // mesh: scale x largest vertex radius, stored by the host
  return fmax(p0, p1);
}

// Cells whose centre lies within `reach` of X along each axis, clipped on
// wall axes (unwrapped coordinates on periodic axes).
__device__ inline void cell_box(const Lattice &L, const double *X, double reach, int *lo, int *hi) {
  const int n[3] = {L.nx, L.ny, L.nz};
  for (int k = 0; k < 3; ++k) {
    const double fa = ceil(X[k] - reach - 0.5), fb = floor(X[k] + reach - 0.5);
    if (!(fa > -1e9 && fb < 1e9)) {
      // a non-finite or runaway centre (a diverged run, already flagged in
      // the status word): an empty box instead of an unbounded cell range
      lo[k] = 0;
      hi[k] = -1;
      continue;
    }
    int a = (int)fa;
    int b = (int)fb;
    if (L.bc[k]) {
      a = max(a, 0);
      b = min(b, n[k] - 1);
    }
    lo[k] = a;
    hi[k] = b;
  }
}

// Coupling box: the cells that can have B > 0 (centre within rc + eps/2).
__device__ inline void particle_boxes(const Lattice &L, DevParticle &p) {
  cell_box(L, p.X, p.rc + 0.5 * L.eps + 1e-9, p.lo, p.hi);
}

__device__ inline void derive(const Lattice &L, DevParticle &p) {
  quat_rot(p.q, p.R);
  p.rc = circumradius(p.shape, p.prm[0], p.prm[1]);
  particle_boxes(L, p);
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
  p.learned = 0;
  derive(L, p);
  out[i] = p;
}

// Mark the particles whose shape family uses its learned indicator (and whose
// aspect matches the trained one).
__global__ void k_mark_learned(DevParticle *parts, int n, LearnedModes modes) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  DevParticle &p = parts[i];
  const double asp = p.prm[1] / p.prm[0];
  int on = 0;
  const int f = p.shape - 1;  // family: rounded cube, spheroid, mesh
  if (f >= 0 && f < 3 && modes.on[f]) on = fabs(asp - modes.aspect[f]) <= 1e-6 * modes.aspect[f];
  // mesh particles always read a distance table: the network's, or the exact one
  p.learned = on ? 1 : (p.shape == 3 ? 2 : 0);
}

__global__ void k_fill_int(int *p, int v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// One thread per (particle, tile of its coupling box): append the particle to
// the tile's list.  grid = (ceil(cap / 64), n).
__global__ void k_bin(Lattice L, const DevParticle *parts, int *tcnt, int *tlist, int *status) {
  const int pid = blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const DevParticle &p = parts[pid];
  int tx[MAX_AXIS_TILES], ty[MAX_AXIS_TILES], tz[MAX_AXIS_TILES];
  const int cx = axis_tiles(p.lo[0], p.hi[0], L.nx, !L.bc[0], TX, tx);
  const int cy = axis_tiles(p.lo[1], p.hi[1], L.ny, !L.bc[1], TY, ty);
  const int cz = axis_tiles(p.lo[2], p.hi[2], L.nz, !L.bc[2], TZ, tz);
  if (k >= cx * cy * cz) return;
  const int a = k % cx, b = (k / cx) % cy, c = k / (cx * cy);
  const int t = tx[a] + L.ntx * (ty[b] + L.nty * tz[c]);
  const int slot = atomicAdd(&tcnt[t], 1);
  if (slot < MAXC) tlist[t * MAXC + slot] = pid;
  else atomicOr(status, ST_TILE_OVERFLOW);
}

// ---------------------------------------------------------------------------
// Fluid -> particle (momentum exchange) and equations of motion
// ---------------------------------------------------------------------------
__device__ inline void cross_sub(const double *a, const double *b, double *o) {
  o[0] -= a[1] * b[2] - a[2] * b[1];
  o[1] -= a[2] * b[0] - a[0] * b[2];
  o[2] -= a[0] * b[1] - a[1] * b[0];
}

// Momentum exchange (Sec. 3.2 MEA, force and torque equations) over the cells
// x_b whose centre is inside the particle, from the stored state of time t in
// pull storage:
//   f_i(x_b + c_i, t) = A[i][x_b],  f_opp(i)(x_b, t) = A[opp i][x_b + c_i],
//   F_h(x_b) = sum_i (c_i - u_p(x_b)) f_i(x_b + c_i) + (c_i + u_p(x_b)) f_opp(i)(x_b)
// (directions whose neighbour lies past a wall are skipped).  The force on the
// particle is -sum F_h, the torque -sum (x_b - X) x F_h.
//
// One workgroup per (particle, slab of a few z-layers of its bounding
// box).  The slab's cells are classified 256 at a time; the inside ones are
// compacted into an LDS queue (in cell order, which keeps the x-runs of a
// convex body contiguous for the loads) and drained 256 at a time, so the 36
// population loads and the FP64 sums run on full wavefronts.  Each thread
// accumulates its cells in queue order; the slab's sum is reduced with a fixed
// wavefront-shuffle tree in FP64 and written as one record.

// A cell of the slab, as box-relative coordinates packed in one int
// (x | y << 8 | z << 16, each < 256), its wrapped lattice coordinates and its
// offset from the particle centre (formed from the unwrapped coordinate, which
// is the minimum image: the box is narrower than half a periodic extent).
struct MeaBox {
  int lo[3], sx, sy, nl;
  double X[3];
};

__device__ inline void mea_cell(const Lattice &L, const MeaBox &g, int packed, int *c, double *d) {
  const int nn[3] = {L.nx, L.ny, L.nz};
  const int r[3] = {packed & 255, (packed >> 8) & 255, packed >> 16};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int u = g.lo[k] + r[k];
    int v = u;
    if (!L.bc[k]) v = v >= nn[k] ? v - nn[k] : (v < 0 ? v + nn[k] : v);
    c[k] = v;
    d[k] = (u + 0.5) - g.X[k];
  }
}

// Population load at a 32-bit byte offset from a wavefront-uniform plane base
// (O32: the host has checked that every offset fits), else 64-bit indexing.
template <bool O32, typename S>
__device__ inline S mea_load(const S *__restrict__ plane, unsigned cell) {
  if constexpr (O32) return *(const S *)((const char *)plane + (cell * (unsigned)sizeof(S)));
  else return plane[cell];
}

// One inside cell's F_h, added as -F_h and -(x_b - X) x F_h.  With the stored
// relative deviations s = K (f - w) / w of f_i(x_b + c_i) and f_opp(i)(x_b):
//   (c - u) f_in + (c + u) f_out = c w (2 + (s_in + s_out) / K) - u w (s_in - s_out) / K,
// so over the kept directions (not past a wall), with w_i = w36_i / 36
// (w36 = 2 along the axes, 1 along the diagonals):
//   F_h = (2 sum c_i w36_i + a / K - u b / K) / 36,
//   a = sum c_i w36_i (s_in + s_out),  b = sum w36_i (s_in - s_out).
// The weight sum is an exact integer (minus the skipped directions' share of
// sum_i c_i w36_i = 0); a and b, sums of the small stored deviations, are
// formed in the arithmetic precision T (FP64 for FP64 storage), and
// everything from them on in FP64.  Cells off the lattice boundary take the
// neighbour index as cell + a constant offset per direction.
template <class ST, bool O32>
__device__ inline void mea_accumulate(const Lattice &L, const typename ST::S *__restrict__ A, const int *c,
                                      const double *d, const double *U, const double *W, double *F, double *T) {
  using S = typename ST::S;
  using TT = typename ST::T;
  const unsigned nxu = (unsigned)L.nx, sxy = (unsigned)L.nx * (unsigned)L.ny;
  const unsigned cell = (unsigned)c[0] + nxu * (unsigned)c[1] + sxy * (unsigned)c[2];
  const bool inner = c[0] > 0 && c[0] < L.nx - 1 && c[1] > 0 && c[1] < L.ny - 1 && c[2] > 0 && c[2] < L.nz - 1;
  int xm = c[0] - 1, xp = c[0] + 1, ym = c[1] - 1, yp = c[1] + 1, zm = c[2] - 1, zp = c[2] + 1;
  bool okxm = true, okxp = true, okym = true, okyp = true, okzm = true, okzp = true;
  if (!inner) {
    xm = c[0] == 0 ? L.nx - 1 : xm; xp = c[0] == L.nx - 1 ? 0 : xp;
    ym = c[1] == 0 ? L.ny - 1 : ym; yp = c[1] == L.ny - 1 ? 0 : yp;
    zm = c[2] == 0 ? L.nz - 1 : zm; zp = c[2] == L.nz - 1 ? 0 : zp;
    okxm = !(L.bc[0] && c[0] == 0); okxp = !(L.bc[0] && c[0] == L.nx - 1);
    okym = !(L.bc[1] && c[1] == 0); okyp = !(L.bc[1] && c[1] == L.ny - 1);
    okzm = !(L.bc[2] && c[2] == 0); okzp = !(L.bc[2] && c[2] == L.nz - 1);
  }
  TT a0 = 0, a1 = 0, a2 = 0, b = 0;
  int k0 = 0, k1 = 0, k2 = 0;  // sum over skipped directions of c_i w36_i
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int w36 = i <= 6 ? 2 : 1;
    unsigned nb;
    bool ok;
    if (inner) {
      nb = cell + (unsigned)(kCX[i] + L.nx * kCY[i] + (int)sxy * kCZ[i]);
      ok = true;
    } else {
      const int ex = kCX[i] == 1 ? xp : (kCX[i] == -1 ? xm : c[0]);
      const int ey = kCY[i] == 1 ? yp : (kCY[i] == -1 ? ym : c[1]);
      const int ez = kCZ[i] == 1 ? zp : (kCZ[i] == -1 ? zm : c[2]);
      ok = (kCX[i] == 1 ? okxp : (kCX[i] == -1 ? okxm : true)) &&
           (kCY[i] == 1 ? okyp : (kCY[i] == -1 ? okym : true)) &&
           (kCZ[i] == 1 ? okzp : (kCZ[i] == -1 ? okzm : true));
      nb = (unsigned)ex + nxu * (unsigned)ey + sxy * (unsigned)ez;
    }
    const S *__restrict__ Ain = A + (size_t)i * (size_t)L.N;
    const S *__restrict__ Aout = A + (size_t)opp(i) * (size_t)L.N;
    const TT sin_ = ST::dec(mea_load<O32>(Ain, cell));
    const TT sout = ST::dec(mea_load<O32>(Aout, nb));
    const TT sp = ok ? sin_ + sout : (TT)0, sm = ok ? sin_ - sout : (TT)0;
    if (kCX[i]) a0 += (TT)(kCX[i] * w36) * sp;
    if (kCY[i]) a1 += (TT)(kCY[i] * w36) * sp;
    if (kCZ[i]) a2 += (TT)(kCZ[i] * w36) * sp;
    b += (TT)w36 * sm;
    if (!ok) { k0 += kCX[i] * w36; k1 += kCY[i] * w36; k2 += kCZ[i] * w36; }
  }
  const double upx = U[0] + W[1] * d[2] - W[2] * d[1];
  const double upy = U[1] + W[2] * d[0] - W[0] * d[2];
  const double upz = U[2] + W[0] * d[1] - W[1] * d[0];
  const double invK = 1.0 / (double)ST::K(), i36 = 1.0 / 36.0;
  const double bk = (double)b * invK;
  // kept directions: sum c w36 = -(skipped share)
  double h[3];
  h[0] = ((double)(-2 * k0) + (double)a0 * invK - upx * bk) * i36;
  h[1] = ((double)(-2 * k1) + (double)a1 * invK - upy * bk) * i36;
  h[2] = ((double)(-2 * k2) + (double)a2 * invK - upz * bk) * i36;
  F[0] -= h[0]; F[1] -= h[1]; F[2] -= h[2];
  cross_sub(d, h, T);
}

// Equations of motion of one particle in FP64 with dt = 1 (Sec. 2.2; Sec. 5.1
// for the external force), from its hydrodynamic force and torque Fs (plus
// the contact force and torque Fc[0..5] when given; Fh and Th record Fs
// alone):
//   U <- U + (F + (m - rho_f V) g) / m;  X <- X + U (wrapped on periodic axes);
//   w_b <- w_b + I^-1 (T_b - w_b x I w_b) in the body frame;
//   q <- normalize(q (x) exp(w_b / 2));  w <- R(q) w_b;
// and the new coupling box.  Particles with m <= 0 are held fixed.
__device__ inline void advance_particle(const Lattice &L, DevParticle &p, const double *Fs, const double *Fc,
                                        int *status) {
  const int nn[3] = {L.nx, L.ny, L.nz};
  for (int k = 0; k < 3; ++k) { p.Fh[k] = Fs[k]; p.Th[k] = Fs[3 + k]; }
  if (p.m > 0.0) {
    const double buoy = p.m - L.rho_f * p.V;
    for (int k = 0; k < 3; ++k) {
      const double Fk = Fc ? Fs[k] + Fc[k] : Fs[k];
      p.U[k] += (Fk + buoy * L.g[k]) / p.m;
      p.X[k] += p.U[k];
      if (!L.bc[k]) {
        if (p.X[k] >= nn[k]) p.X[k] -= nn[k];
        else if (p.X[k] < 0.0) p.X[k] += nn[k];
        if (!(p.X[k] >= 0.0 && p.X[k] < nn[k])) {
          // moved a lattice length or more in one step, or non-finite: the
          // run has diverged; keep the centre inside the lattice
          atomicOr(status, ST_UNSTABLE);
          p.X[k] = 0.5 * nn[k];
        }
      } else if (!(p.X[k] >= 0.0 && p.X[k] <= nn[k])) {
        atomicOr(status, ST_WALL_EXIT);
      }
    }
    const double *R = p.R;
    double wb[3], tb[3];
    for (int k = 0; k < 3; ++k) {
      wb[k] = R[0 * 3 + k] * p.W[0] + R[1 * 3 + k] * p.W[1] + R[2 * 3 + k] * p.W[2];
      tb[k] = Fc ? R[0 * 3 + k] * (Fs[3] + Fc[3]) + R[1 * 3 + k] * (Fs[4] + Fc[4]) + R[2 * 3 + k] * (Fs[5] + Fc[5])
                 : R[0 * 3 + k] * Fs[3] + R[1 * 3 + k] * Fs[4] + R[2 * 3 + k] * Fs[5];
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
    const double qn[4] = {q[0] * d0 - q[1] * d1 - q[2] * d2 - q[3] * d3,
                          q[0] * d1 + q[1] * d0 + q[2] * d3 - q[3] * d2,
                          q[0] * d2 - q[1] * d3 + q[2] * d0 + q[3] * d1,
                          q[0] * d3 + q[1] * d2 - q[2] * d1 + q[3] * d0};
    const double nq = sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
    for (int k = 0; k < 4; ++k) p.q[k] = qn[k] / nq;
    quat_rot(p.q, p.R);
    for (int k = 0; k < 3; ++k)
      p.W[k] = p.R[k * 3 + 0] * wb[0] + p.R[k * 3 + 1] * wb[1] + p.R[k * 3 + 2] * wb[2];
    if (!(p.X[0] == p.X[0] && p.X[1] == p.X[1] && p.X[2] == p.X[2])) atomicOr(status, ST_UNSTABLE);
    particle_boxes(L, p);
  }
}

// Number of slabs of `layers` z-layers of a momentum-exchange box (at least
// one: an empty box still writes a zero record).
__device__ inline int mea_slabs(int lo2, int hi2, int layers) {
  return hi2 < lo2 ? 1 : (hi2 - lo2 + layers) / layers;
}

// Momentum exchange of one slab: one workgroup per (particle, slab) reduces the slab's
// inside cells into one record partial[pid][slab][F, T].  The slab is
// classified in rounds: each wavefront takes 64 / sx whole x-rows (lane ->
// (x, row)), the inside cells are compacted into the LDS queue, and full
// queues of 256 cells are drained by all threads at once.
template <class ST, bool O32>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ST::kind == 2 ? 4 : 3))) void k_mea(Lattice L, const typename ST::S *__restrict__ A,
                                             const DevParticle *__restrict__ parts, const int *__restrict__ order,
                                             int n, int lmax, int layers, int chunked,
                                             double *__restrict__ partial) {
  __shared__ int queue[512];
  __shared__ int wcnt[4];
  __shared__ double red[4][6];
  // work item -> (particle rank in `order`, slab): slab-major (every
  // particle's first slab, then every second slab, ...), or with `chunked`
  // the slabs of one particle consecutive and each XCD on a contiguous run of
  // the order (shared rows read through one L2: pays where the exchange is
  // bound by HBM traffic, i.e. for many particles)
  const int nslot = (lmax + layers - 1) / layers;
  int rank, slab;
  if (chunked) {
    const int item = xcd_chunk(blockIdx.x, n * nslot);
    rank = item / nslot;
    slab = item - rank * nslot;
  } else {
    slab = blockIdx.x / n;
    rank = blockIdx.x - slab * n;
  }
  const int pid = order[rank];
  const DevParticle &sp = parts[pid];
  MeaBox g;
  int hi[3];
  cell_box(L, sp.X, sp.rc + 1e-9, g.lo, hi);
  const int nslab = mea_slabs(g.lo[2], hi[2], layers);
  if (slab >= nslab) return;   // uniform per workgroup
  g.lo[2] += slab * layers;
  g.sx = hi[0] - g.lo[0] + 1;
  g.sy = hi[1] - g.lo[1] + 1;
  g.nl = min(layers, hi[2] - g.lo[2] + 1);
  for (int k = 0; k < 3; ++k) g.X[k] = sp.X[k];
  const int shape = sp.shape;
  const double p0 = sp.prm[0], p1 = sp.prm[1];
  const double U[3] = {sp.U[0], sp.U[1], sp.U[2]};
  const double W[3] = {sp.W[0], sp.W[1], sp.W[2]};
  double R[9];
  for (int k = 0; k < 9; ++k) R[k] = sp.R[k];
  const int learned = sp.learned && L.tables;
  const int tsx = sp.hi[0] - sp.lo[0] + 1, tsy = sp.hi[1] - sp.lo[1] + 1;
  const int t = threadIdx.x, w = wave_id(), lane = lane_id();
  const int rows = (g.sx > 0 && g.sy > 0 && g.nl > 0) ? g.sy * g.nl : 0;  // sx <= 64 (host check)
  const int sxp = rows > 0 ? g.sx : 64;
  const int rpw = 64 / sxp;     // rows per wavefront and round
  const int rx = lane % sxp, rsub = lane / sxp;
  double F[3] = {0, 0, 0}, T[3] = {0, 0, 0};
  int queued = 0;  // uniform
  for (int r0 = 0; r0 < rows; r0 += 4 * rpw) {
    const int row = r0 + w * rpw + rsub;
    bool in = false;
    int packed = 0;
    if (rsub < rpw && row < rows) {
      const int ry = row % g.sy, rz = row / g.sy;
      packed = rx | (ry << 8) | (rz << 16);
      int c[3];
      double d[3];
      mea_cell(L, g, packed, c, d);
      if (learned) {
        const int lx = g.lo[0] + rx - sp.lo[0], ly = g.lo[1] + ry - sp.lo[1], lz = g.lo[2] + rz - sp.lo[2];
        in = L.tables[(size_t)pid * L.table_cap + lx + tsx * (ly + tsy * lz)] <= 0.0f;
      } else {
        double b[3] = {d[0], d[1], d[2]};
        if (shape != 0) {
          b[0] = R[0] * d[0] + R[3] * d[1] + R[6] * d[2];
          b[1] = R[1] * d[0] + R[4] * d[1] + R[7] * d[2];
          b[2] = R[2] * d[0] + R[5] * d[1] + R[8] * d[2];
        }
        in = inside_body(shape, p0, p1, b[0], b[1], b[2]);
      }
    }
    const unsigned long long mask = __ballot(in);
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wcnt[w] = __popcll(mask);
    __syncthreads();
    int off = queued, added = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      off += (k < w) ? wcnt[k] : 0;
      added += wcnt[k];
    }
    if (in) queue[off + before] = packed;
    queued += added;
    __syncthreads();
    if (queued >= 256) {
      int c[3];
      double d[3];
      mea_cell(L, g, queue[t], c, d);
      mea_accumulate<ST, O32>(L, A, c, d, U, W, F, T);
      const int rest = queued - 256;
      const int keep = t < rest ? queue[256 + t] : 0;
      __syncthreads();
      if (t < rest) queue[t] = keep;
      queued = rest;
      __syncthreads();
    }
  }
  if (t < queued) {
    int c[3];
    double d[3];
    mea_cell(L, g, queue[t], c, d);
    mea_accumulate<ST, O32>(L, A, c, d, U, W, F, T);
  }
  double v[6] = {F[0], F[1], F[2], T[0], T[1], T[2]};
#pragma unroll
  for (int k = 0; k < 6; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) red[w][k] = v[k];
  }
  __syncthreads();
  if (t < 6) partial[((size_t)pid * lmax + slab) * 6 + t] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
}

// Sphere contact (an addition: the paper runs without a contact model and
// cites one, Sec. 2.2, 3.2 and 5.3): the short-range repulsion of Glowinski et al.
// (J. Comput. Phys. 169, 2001).  Spheres p and q with centre distance
// d < R_p + R_q + range (minimum image on periodic axes) repel along the line
// of centres with k ((R_p + R_q + range - d) / range)^2.
//
// Pair search on a uniform grid of the particle centres (from
// CONTACT_GRID_MIN particles on; below, k_contact_pairs): cells at least the
// largest pair reach 2 w_max + range wide on every axis (w = R for spheres,
// the circumradius otherwise), so the partners of p lie in the 27 cells
// around p's cell (fewer where an axis has one or two cells; no wrap across
// walls).  The grid is a counting sort: k_cgrid_count counts the centres per
// cell (and stores each centre with w), k_cgrid_scan turns the counts into
// cell starts, k_cgrid_fill places the particle indices (in no fixed order
// within a cell).  k_contact then lists, per particle, the partners whose
// bounding spheres come within the range (at most CONTACT_CAND; more is
// reported as ST_CONTACT_OVERFLOW), ranks them by index, sums the sphere
// pairs' forces into out[p] and copies the pairs with a non-spherical
// particle into cand[p] / ccnt[p] for k_contact_shapes.  The sums and lists
// are independent of the order within the cells.
__device__ inline int cgrid_axis(double x, double size, int g) {
  double q = x / size;
  if (!(q >= 0.0)) q = 0.0;  // also a non-finite centre
  if (q > (double)(g - 1)) q = (double)(g - 1);
  return (int)q;
}

__global__ __launch_bounds__(256) void k_cgrid_count(const DevParticle *__restrict__ parts, int n, ContactGrid cg,
                                                     int *__restrict__ gcount, int *__restrict__ gcell,
                                                     double4 *__restrict__ gpos) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const DevParticle &P = parts[p];
  const double *X = P.X;
  const int cell = cgrid_axis(X[0], cg.size[0], cg.g[0]) +
                   cg.g[0] * (cgrid_axis(X[1], cg.size[1], cg.g[1]) + cg.g[1] * cgrid_axis(X[2], cg.size[2], cg.g[2]));
  gcell[p] = cell;
  // centre and w = R for spheres, -circumradius otherwise
  gpos[p] = make_double4(X[0], X[1], X[2], P.shape == 0 ? P.prm[0] : -P.rc);
  atomicAdd(&gcount[cell], 1);
}

// One 1024-thread workgroup: gcount[0 .. ncells) -> exclusive starts in
// gcount (gcount[ncells] = n) and the same starts in gfill (the insertion
// pointers of k_cgrid_fill).
__global__ __launch_bounds__(1024) void k_cgrid_scan(int *__restrict__ gcount, int ncells,
                                                     int *__restrict__ gfill) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int per = (ncells + 1023) / 1024;
  const int b = min(ncells, t * per), e = min(ncells, b + per);
  int sum = 0;
  for (int c = b; c < e; ++c) sum += gcount[c];
  part[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele scan
    const int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - sum;  // exclusive prefix of this thread's range
  for (int c = b; c < e; ++c) {
    const int v = gcount[c];
    gcount[c] = run;
    gfill[c] = run;
    run += v;
  }
  if (t == 1023) gcount[ncells] = part[1023];
}

__global__ __launch_bounds__(256) void k_cgrid_fill(int n, const int *__restrict__ gcell, int *__restrict__ gfill,
                                                    int *__restrict__ glist) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  glist[atomicAdd(&gfill[gcell[p]], 1)] = p;
}

// distinct grid cells next to cell c on an axis of g cells (wrapped on a
// periodic axis, clipped at walls); returns their count
__device__ inline int cgrid_near(int c, int g, bool periodic, int *out) {
  if (g <= 2 && periodic) {
    for (int k = 0; k < g; ++k) out[k] = k;
    return g;
  }
  int m = 0;
  for (int d = -1; d <= 1; ++d) {
    int v = c + d;
    if (periodic) v = v < 0 ? v + g : (v >= g ? v - g : v);
    else if (v < 0 || v >= g) continue;
    out[m++] = v;
  }
  return m;
}

// One wavefront per particle p (four per workgroup): the members of the
// cells around p's cell are enumerated as one flat list spread over the
// lanes, the partners within the range compacted in LDS, ranked by index,
// and then summed (sphere pairs, fixed wavefront tree) or copied to
// cand[p] in increasing index (pairs with a non-spherical particle).
__global__ __launch_bounds__(256) void k_contact(Lattice L, int n, ContactParams c, ContactGrid cg,
                                                 const double4 *__restrict__ gpos, const int *__restrict__ gstart,
                                                 const int *__restrict__ gcell, const int *__restrict__ glist,
                                                 double *__restrict__ out, int *__restrict__ cand,
                                                 int *__restrict__ ccnt, int *status) {
  __shared__ int cbeg[4][28], cpre[4][28];
  __shared__ int found[4][CONTACT_CAND], sorted[4][CONTACT_CAND];
  const int w = wave_id(), lane = lane_id();
  const int p = blockIdx.x * 4 + w;
  if (p >= n) return;  // uniform per wavefront; no workgroup barrier below
  const int nn[3] = {L.nx, L.ny, L.nz};
  const double4 P = gpos[p];
  const int cell = gcell[p];
  const int cc[3] = {cell % cg.g[0], (cell / cg.g[0]) % cg.g[1], cell / (cg.g[0] * cg.g[1])};
  int near[3][3], nnear[3];
  for (int a = 0; a < 3; ++a) nnear[a] = cgrid_near(cc[a], cg.g[a], !L.bc[a], near[a]);
  const int ncell = nnear[0] * nnear[1] * nnear[2];
  // members of the neighbouring cells: counts, then their running offsets
  int cnt_c = 0, beg_c = 0;
  if (lane < ncell) {
    const int ix = lane % nnear[0], iy = (lane / nnear[0]) % nnear[1], iz = lane / (nnear[0] * nnear[1]);
    const int q_cell = near[0][ix] + cg.g[0] * (near[1][iy] + cg.g[1] * near[2][iz]);
    beg_c = gstart[q_cell];
    cnt_c = gstart[q_cell + 1] - beg_c;
  }
  int pre = cnt_c;  // inclusive prefix over the lanes
  for (int off = 1; off < 32; off <<= 1) {
    const int v = __shfl_up(pre, off, 64);
    if (lane >= off) pre += v;
  }
  const int total = __shfl(pre, 31, 64);
  if (lane < 28) {
    cbeg[w][lane] = beg_c;
    cpre[w][lane] = pre - cnt_c;
  }
  __builtin_amdgcn_wave_barrier();
  int nfound = 0;
  bool over = false;
  for (int i0 = 0; i0 < total; i0 += 64) {
    const int i = i0 + lane;
    bool in = false;
    int q = 0;
    if (i < total) {
      int j = 0;
      while (j + 1 < ncell && cpre[w][j + 1] <= i) ++j;
      q = glist[cbeg[w][j] + (i - cpre[w][j])];
      if (q != p) {
        const double4 Q = gpos[q];
        const double Qx[3] = {Q.x, Q.y, Q.z}, Px[3] = {P.x, P.y, P.z};
        double d2 = 0.0;
        for (int a = 0; a < 3; ++a) {
          double dx = Px[a] - Qx[a];
          if (!L.bc[a]) dx = dx > 0.5 * nn[a] ? dx - nn[a] : (dx < -0.5 * nn[a] ? dx + nn[a] : dx);
          d2 += dx * dx;
        }
        const double reach = fabs(P.w) + fabs(Q.w) + c.range;
        in = d2 < reach * reach && d2 != 0.0;
      }
    }
    const unsigned long long mask = __ballot(in);
    const int slot = nfound + __popcll(mask & ((1ull << lane) - 1ull));
    if (in) {
      if (slot < CONTACT_CAND) found[w][slot] = q;
      else over = true;
    }
    nfound += __popcll(mask);
  }
  if (__ballot(over)) {
    if (lane == 0) atomicOr(status, ST_CONTACT_OVERFLOW);
  }
  const int np = min(nfound, CONTACT_CAND);
  __builtin_amdgcn_wave_barrier();
  // rank by index
  if (lane < np) {
    const int v = found[w][lane];
    int rank = 0;
    for (int k = 0; k < np; ++k) rank += found[w][k] < v;
    sorted[w][rank] = v;
  }
  __builtin_amdgcn_wave_barrier();
  double f[3] = {0.0, 0.0, 0.0};
  bool shape_pair = false;
  int q = -1;
  if (lane < np) {
    q = sorted[w][lane];
    const double4 Q = gpos[q];
    if (P.w > 0.0 && Q.w > 0.0) {
      const double Qx[3] = {Q.x, Q.y, Q.z}, Px[3] = {P.x, P.y, P.z};
      double dx[3];
      for (int a = 0; a < 3; ++a) {
        dx[a] = Px[a] - Qx[a];
        if (!L.bc[a]) dx[a] = dx[a] > 0.5 * nn[a] ? dx[a] - nn[a] : (dx[a] < -0.5 * nn[a] ? dx[a] + nn[a] : dx[a]);
      }
      const double d = sqrt(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
      const double sc = (P.w + Q.w + c.range - d) / c.range;
      for (int a = 0; a < 3; ++a) f[a] = c.k * sc * sc * dx[a] / d;
    } else {
      shape_pair = c.k != 0.0;
    }
  }
  const unsigned long long smask = __ballot(shape_pair);
  if (shape_pair) cand[(size_t)p * CONTACT_CAND + __popcll(smask & ((1ull << lane) - 1ull))] = q;
  for (int a = 0; a < 3; ++a) f[a] = wave_sum(f[a]);
  if (lane == 0) {
    ccnt[p] = __popcll(smask);
    for (int a = 0; a < 3; ++a) out[(size_t)p * 3 + a] = f[a];
  }
}

// Pair search without a grid, for fewer than CONTACT_GRID_MIN particles
// (where the grid's extra launches and dependent loads cost more than the
// n^2 tests): workgroup (bp, c) takes 256 particles p and the c-th of up to
// 64 contiguous chunks of partners q (enough workgroups to fill the chip for
// a few hundred particles), staged in LDS 1024 at a time as (X, w); each
// thread sums its chunk in increasing q into out[c][p].  Pairs with a
// non-spherical particle are appended to cand[p] / ccnt[p] in no fixed order
// (k_contact_shapes sorts them).
__global__ __launch_bounds__(256) void k_contact_pairs(Lattice L, const DevParticle *__restrict__ parts, int n,
                                                 ContactParams c, double *__restrict__ out, int *__restrict__ cand,
                                                 int *__restrict__ ccnt, int *status) {
  __shared__ double4 sq[CONTACT_TILE];
  const int nchunk = gridDim.y;
  const int per = (n + nchunk - 1) / nchunk;
  const int q_begin = blockIdx.y * per, q_end = min(n, q_begin + per);
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int nn[3] = {L.nx, L.ny, L.nz};
  double Xp[3] = {0, 0, 0}, wp = 0.0;
  if (p < n) {
    for (int a = 0; a < 3; ++a) Xp[a] = parts[p].X[a];
    wp = parts[p].shape == 0 ? parts[p].prm[0] : -parts[p].rc;
  }
  double acc[3] = {0.0, 0.0, 0.0};
  for (int t0 = q_begin; t0 < q_end; t0 += CONTACT_TILE) {
    const int nt = min(CONTACT_TILE, q_end - t0);
    __syncthreads();
    for (int j = threadIdx.x; j < nt; j += blockDim.x) {
      const DevParticle &q = parts[t0 + j];
      sq[j] = make_double4(q.X[0], q.X[1], q.X[2], q.shape == 0 ? q.prm[0] : -q.rc);
    }
    __syncthreads();
    if (p < n) {
      for (int j = 0; j < nt; ++j) {
        const double4 v = sq[j];
        if (t0 + j == p) continue;
        double dx[3] = {Xp[0] - v.x, Xp[1] - v.y, Xp[2] - v.z};
        for (int a = 0; a < 3; ++a)  // minimum image (centres lie in [0, n) on periodic axes)
          if (!L.bc[a]) dx[a] = dx[a] > 0.5 * nn[a] ? dx[a] - nn[a] : (dx[a] < -0.5 * nn[a] ? dx[a] + nn[a] : dx[a]);
        const double reach = fabs(wp) + fabs(v.w) + c.range;
        const double d2 = dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2];
        if (!(d2 < reach * reach) || d2 == 0.0) continue;
        if (wp > 0.0 && v.w > 0.0) {
          const double d = sqrt(d2);
          const double sc = (reach - d) / c.range;
          for (int a = 0; a < 3; ++a) acc[a] += c.k * sc * sc * dx[a] / d;
        } else if (c.k != 0.0) {
          const int slot = atomicAdd(&ccnt[p], 1);
          if (slot < CONTACT_CAND) cand[(size_t)p * CONTACT_CAND + slot] = t0 + j;
          else atomicOr(status, ST_CONTACT_OVERFLOW);
        }
      }
    }
  }
  if (p < n)
    for (int a = 0; a < 3; ++a) out[((size_t)blockIdx.y * n + p) * 3 + a] = acc[a];
}

// Wall part of the contact force on sphere p, added to Fc: each wall acts as
// the mirror image (centre distance 2 h from the image; pushes away from the
// wall with kw ((2 R + range - 2 h) / range)^2), axis by axis, lower wall
// first.
__device__ inline void contact_walls(const Lattice &L, const DevParticle &p, const ContactParams &c, double *Fc) {
  if (p.shape != 0) return;
  const int nn[3] = {L.nx, L.ny, L.nz};
  const double reach = 2.0 * p.prm[0] + c.range;
  for (int a = 0; a < 3; ++a) {
    if (!L.bc[a]) continue;
    const double dlo = 2.0 * p.X[a], dhi = 2.0 * (nn[a] - p.X[a]);
    if (dlo < reach) {
      const double sc = (reach - dlo) / c.range;
      Fc[a] += c.kw * sc * sc;
    }
    if (dhi < reach) {
      const double sc = (reach - dhi) / c.range;
      Fc[a] -= c.kw * sc * sc;
    }
  }
}

// One 64-thread workgroup per particle: the slab records of k_mea summed in a
// fixed order (thread t takes slabs t, t + 64, ..., then a fixed wavefront
// butterfly), the equations of motion, then the particle appended to the tile
// lists of its new coupling box.
template <bool CONTACT>
__global__ __launch_bounds__(64) void k_eom_bin(Lattice L, DevParticle *__restrict__ parts, int n, int lmax,
                                                int layers, const double *__restrict__ partial, ContactParams c,
                                                const double *__restrict__ contact,
                                                const double *__restrict__ shapes, int *tcnt, int *tlist,
                                                int *status) {
  __shared__ int ts[3][MAX_AXIS_TILES];
  __shared__ int tn[3];
  const int pid = blockIdx.x;
  const int t = threadIdx.x;
  // the slab records are loaded before their count is known (every slot up
  // to the largest count exists), so the loads overlap the box computation
  const double *src = partial + (size_t)pid * lmax * 6;
  const int nmax = (lmax + layers - 1) / layers;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  double first[6];
  const bool have = t < nmax;
  if (have)
    for (int k = 0; k < 6; ++k) first[k] = src[t * 6 + k];
  // contact: lane b holds record b of the particle (contact_chunks(n) of
  // them below CONTACT_GRID_MIN particles, else one), reduced by the fixed
  // wavefront tree
  double fc[3] = {0.0, 0.0, 0.0};
  if (CONTACT && t < contact_chunks(n))
    for (int a = 0; a < 3; ++a) fc[a] = contact[((size_t)t * n + pid) * 3 + a];
  int lo[3], hi[3];
  cell_box(L, parts[pid].X, parts[pid].rc + 1e-9, lo, hi);
  const int nrec = mea_slabs(lo[2], hi[2], layers);
  if (have && t < nrec)
    for (int k = 0; k < 6; ++k) acc[k] = first[k];
  for (int r = t + 64; r < nrec; r += 64)
    for (int k = 0; k < 6; ++k) acc[k] += src[r * 6 + k];
  for (int k = 0; k < 6; ++k) acc[k] = wave_sum(acc[k]);
  if (CONTACT)
    for (int a = 0; a < 3; ++a) fc[a] = wave_sum(fc[a]);
  if (t == 0) {
    DevParticle p = parts[pid];
    if (CONTACT) {
      contact_walls(L, p, c, fc);
      double fct[6] = {fc[0], fc[1], fc[2], 0.0, 0.0, 0.0};
      if (shapes)
        for (int k = 0; k < 6; ++k) fct[k] += shapes[(size_t)pid * 6 + k];
      advance_particle(L, p, acc, fct, status);
    } else {
      advance_particle(L, p, acc, nullptr, status);
    }
    parts[pid] = p;
    tn[0] = axis_tiles(p.lo[0], p.hi[0], L.nx, !L.bc[0], TX, ts[0]);
    tn[1] = axis_tiles(p.lo[1], p.hi[1], L.ny, !L.bc[1], TY, ts[1]);
    tn[2] = axis_tiles(p.lo[2], p.hi[2], L.nz, !L.bc[2], TZ, ts[2]);
  }
  __syncthreads();
  const int cx = tn[0], cy = tn[1], cz = tn[2];
  for (int k = t; k < cx * cy * cz; k += 64) {
    const int a = k % cx, b = (k / cx) % cy, c = k / (cx * cy);
    const int tile = ts[0][a] + L.ntx * (ts[1][b] + L.nty * ts[2][c]);
    const int slot = atomicAdd(&tcnt[tile], 1);
    if (slot < MAXC) tlist[tile * MAXC + slot] = pid;
    else atomicOr(status, ST_TILE_OVERFLOW);
  }
}

// ---------------------------------------------------------------------------
// Contact of non-spherical particles (an addition, like the sphere contact
// above): the sphere repulsion written as a volume law on surface nodes.
// Both bodies grown by zeta/2 overlap in about
//   V = 1/2 (sum_{s in P} a_s delta_Q(s) + sum_{s in Q} a_s delta_P(s)),
// delta_Q(s) = max(0, zeta - d_Q(s)) for a surface node s of P; the force
// on P is K = k / (pi R_eff zeta^2) times the node sums with the partner's
// outward normal grad d:
//   F_P = K [ sum_{s in P} 1/2 a_s delta_Q(s) grad d_Q(s)
//           - sum_{s in Q} 1/2 a_s delta_P(s) grad d_P(s) ],
//   T_P = the same sums of (s - X_P) x (...),
// R_eff = R_P R_Q / (R_P + R_Q) with volume-equivalent radii (for two
// spheres this is the sphere law to leading order in the penetration); a
// wall acts as the mirror image: delta = zeta - 2 h_s, K_w = k_w / (pi R_P / 2
// zeta^2), no factor 1/2, along the wall normal.  Nodes: CONTACT_NODES
// Fibonacci directions u_m (a table in the workspace), the surface point on
// the ray from the centre in closed form (sphere, spheroid, rounded cube) or
// by the nearest triangle hit (mesh), area weight a = (4 pi / M) t^2 /
// (u . n).  Pairs of two spheres are left to k_contact.
//
// One wavefront per particle p: the partners (bounding spheres within the
// range, listed by k_contact; taken in increasing index; pairs that the
// support functions separate by the range along the line of centres are
// skipped) and then the walls; for each, the nodes whose ray segment between
// the inscribed and the circumscribed radius comes within reach are
// compacted in LDS and evaluated 64 at a time.  Per-lane FP64 sums, one
// fixed wavefront reduction at the end: record shapes[p] = (F, T).
// ---------------------------------------------------------------------------
__device__ inline double inscribed_radius(const DevParticle &P) {
  return P.shape == 2 ? fmin(P.prm[0], P.prm[1]) : (P.shape == 3 ? P.prm[2] : P.prm[0]);
}

template <bool MESH>
__device__ inline double body_sdf(const Lattice &L, const DevParticle &P, const double *y) {
  if (MESH && P.shape == 3) return mesh_sdf<double>(L.mesh, L.mesh_nt, P.prm[0], y[0], y[1], y[2]);
  return sdf_body<double>(P.shape, P.prm[0], P.prm[1], y[0], y[1], y[2]);
}

// Nearest point (x0, x1) to (y0, y1) >= 0 on the ellipse (u/e0)^2 + (v/e1)^2
// = 1, e0 >= e1: the same monotone Newton iteration for the Lagrange root t,
// with the same operations, as the distance function of the coupling, so
// that |(x0, x1) - (y0, y1)| is that distance bit for bit.
__device__ inline void ellipse_nearest(double e0, double e1, double y0, double y1, double &x0, double &x1) {
  const double e0s = e0 * e0, e1s = e1 * e1;
  if (y1 > 0.0) {
    if (y0 > 0.0) {
      const double a = e0 * y0, b = e1 * y1, lo = b - e1s;
      double t = 0.0;
      for (int it = 0; it < 100; ++it) {
        const double i0 = 1.0 / (t + e0s), i1 = 1.0 / (t + e1s);
        const double r0 = a * i0, r1 = b * i1;
        const double gv = r0 * r0 + r1 * r1 - 1.0;
        const double dg = -2.0 * (r0 * r0 * i0 + r1 * r1 * i1);
        double tn = t - gv * (1.0 / dg);
        if (tn < lo) tn = lo;
        if (it > 0 && !(tn > t)) break;
        t = tn;
      }
      x0 = e0s * y0 / (t + e0s);
      x1 = e1s * y1 / (t + e1s);
    } else {
      x0 = 0.0;
      x1 = e1;
    }
    return;
  }
  const double den = e0s - e1s;
  if (e0 * y0 < den) {
    x0 = e0s * y0 / den;
    const double s = x0 / e0;
    x1 = e1 * sqrt(fmax(0.0, 1.0 - s * s));
  } else {
    x0 = e0;
    x1 = 0.0;
  }
}

// Signed distance of the spheroid (symmetry axis body x with semi-axis a,
// radial semi-axis b) at the body-frame point y, and its unit gradient: the
// ellipse normal at the nearest point of the meridian plane.  The distance
// equals the coupling's spheroid distance bit for bit.
__device__ inline double spheroid_distance_normal(double a, double b, const double *y, double *g) {
  const double y0 = fabs(y[0]), r = sqrt(y[1] * y[1] + y[2] * y[2]);
  double x0, x1;
  if (a >= b) ellipse_nearest(a, b, y0, r, x0, x1);
  else ellipse_nearest(b, a, r, y0, x1, x0);
  const double d = a >= b ? sqrt((x0 - y0) * (x0 - y0) + (x1 - r) * (x1 - r))
                          : sqrt((x1 - r) * (x1 - r) + (x0 - y0) * (x0 - y0));
  const double n0 = x0 / (a * a), n1 = x1 / (b * b);
  const double nn = 1.0 / sqrt(n0 * n0 + n1 * n1);
  g[0] = copysign(n0 * nn, y[0]);
  if (r > 0.0) {
    g[1] = n1 * nn * y[1] / r;
    g[2] = n1 * nn * y[2] / r;
  } else {  // on the axis: the nearest points form a ring; one of them
    g[1] = n1 * nn;
    g[2] = 0.0;
  }
  const double k = (y[0] * y[0]) / (a * a) + (y[1] * y[1] + y[2] * y[2]) / (b * b);
  return k <= 1.0 ? -d : d;
}

// Unit gradient of the body-frame signed distance at y: the outward normal
// at the nearest surface point.  Closed forms for the sphere, the rounded
// cube (the dilation direction outside the core, the axis of the nearest face
// inside it) and the spheroid (the ellipse normal at the nearest point of the
// meridian plane); central differences (step 1e-5) for a mesh.
template <bool MESH>
__device__ inline void body_sdf_normal(const Lattice &L, const DevParticle &P, const double *y, double *g) {
  if (P.shape == 0) {
    const double r = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    if (r > 0.0) {
      for (int k = 0; k < 3; ++k) g[k] = y[k] / r;
    } else {
      g[0] = 1.0; g[1] = g[2] = 0.0;
    }
    return;
  }
  if (P.shape == 1) {
    const double c = P.prm[0] - P.prm[1];
    double q[3], o[3], on = 0.0;
    for (int k = 0; k < 3; ++k) {
      q[k] = fabs(y[k]) - c;
      o[k] = fmax(q[k], 0.0);
      on += o[k] * o[k];
    }
    if (on > 0.0) {
      on = 1.0 / sqrt(on);
      for (int k = 0; k < 3; ++k) g[k] = copysign(o[k] * on, y[k]);
    } else {
      const int m = q[0] >= q[1] && q[0] >= q[2] ? 0 : (q[1] >= q[2] ? 1 : 2);
      for (int k = 0; k < 3; ++k) g[k] = k == m ? copysign(1.0, y[k]) : 0.0;
    }
    return;
  }
  if (P.shape == 2) {
    spheroid_distance_normal(P.prm[0], P.prm[1], y, g);
    return;
  }
  const double h = 1e-5;
  double dv[6];
#pragma unroll 1
  for (int j = 0; j < 6; ++j) {  // one distance evaluation in the loop body
    double yj[3] = {y[0], y[1], y[2]};
    yj[j >> 1] += (j & 1) ? -h : h;
    dv[j] = body_sdf<MESH>(L, P, yj);
  }
  double nn = 0.0;
  for (int k = 0; k < 3; ++k) {
    g[k] = (dv[2 * k] - dv[2 * k + 1]) / (2.0 * h);
    nn += g[k] * g[k];
  }
  nn = 1.0 / sqrt(nn);
  for (int k = 0; k < 3; ++k) g[k] *= nn;
}

// Surface point t u on the ray from the centre along the unit body direction
// u, and the outward body normal n there.
template <bool MESH>
__device__ inline double surface_ray(const Lattice &L, const DevParticle &P, const double *u, double *n) {
  if (P.shape == 0) {
    for (int k = 0; k < 3; ++k) n[k] = u[k];
    return P.prm[0];
  }
  if (P.shape == 2) {  // spheroid: semi-axis a along body x, b along y and z
    const double ia2 = 1.0 / (P.prm[0] * P.prm[0]), ib2 = 1.0 / (P.prm[1] * P.prm[1]);
    const double t = 1.0 / sqrt(u[0] * u[0] * ia2 + (u[1] * u[1] + u[2] * u[2]) * ib2);
    const double g[3] = {t * u[0] * ia2, t * u[1] * ib2, t * u[2] * ib2};
    const double gn = 1.0 / sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    for (int k = 0; k < 3; ++k) n[k] = g[k] * gn;
    return t;
  }
  if (P.shape == 1) {
    // rounded cube of half-size h and corner radius r around the core cube
    // [-c, c]^3, c = h - r: t|u| lies at distance r from the core; the hit is
    // on a face, an edge or a corner piece (one, two or three coordinates
    // beyond c), tried in that order
    const double h = P.prm[0], r = P.prm[1], c = h - r;
    double v[3] = {fabs(u[0]), fabs(u[1]), fabs(u[2])};
    double v1 = fmax(v[0], fmax(v[1], v[2])), v3 = fmin(v[0], fmin(v[1], v[2]));
    const double v2 = v[0] + v[1] + v[2] - v1 - v3;
    double t = (c + r) / v1;
    if (t * v2 > c) {
      const double A = v1 * v1 + v2 * v2, B = c * (v1 + v2);
      t = (B + sqrt(fmax(0.0, B * B - A * (2.0 * c * c - r * r)))) / A;
      if (t * v3 > c) {
        const double S = v1 + v2 + v3;
        t = c * S + sqrt(fmax(0.0, c * c * S * S - 3.0 * c * c + r * r));
      }
    }
    double o[3], on = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double b = t * u[k];
      o[k] = b - fmin(fmax(b, -c), c);
      on += o[k] * o[k];
    }
    if (on > 0.0) {
      on = 1.0 / sqrt(on);
      for (int k = 0; k < 3; ++k) n[k] = o[k] * on;
    } else {  // sharp cube face: the axis of the largest coordinate
      const int a = v[0] >= v[1] && v[0] >= v[2] ? 0 : (v[1] >= v[2] ? 1 : 2);
      for (int k = 0; k < 3; ++k) n[k] = k == a ? (u[k] >= 0.0 ? 1.0 : -1.0) : 0.0;
    }
    return t;
  }
  // mesh (scale prm[0]): nearest triangle hit of the ray from the centre
  // (Moller-Trumbore), normal of that triangle
  if (!MESH) {
    for (int k = 0; k < 3; ++k) n[k] = u[k];
    return P.rc;
  }
  double best = 1e300;
  n[0] = u[0]; n[1] = u[1]; n[2] = u[2];
  const double sc = P.prm[0];
  for (int tr = 0; tr < L.mesh_nt; ++tr) {
    const float4 A = L.mesh[3 * tr], Bv = L.mesh[3 * tr + 1], Cv = L.mesh[3 * tr + 2];
    const double a[3] = {sc * A.x, sc * A.y, sc * A.z};
    const double e1[3] = {sc * Bv.x - a[0], sc * Bv.y - a[1], sc * Bv.z - a[2]};
    const double e2[3] = {sc * Cv.x - a[0], sc * Cv.y - a[1], sc * Cv.z - a[2]};
    const double pv[3] = {u[1] * e2[2] - u[2] * e2[1], u[2] * e2[0] - u[0] * e2[2], u[0] * e2[1] - u[1] * e2[0]};
    const double det = e1[0] * pv[0] + e1[1] * pv[1] + e1[2] * pv[2];
    if (fabs(det) < 1e-300) continue;
    const double id = 1.0 / det;
    const double tv[3] = {-a[0], -a[1], -a[2]};
    const double bu = (tv[0] * pv[0] + tv[1] * pv[1] + tv[2] * pv[2]) * id;
    if (bu < 0.0 || bu > 1.0) continue;
    const double qv[3] = {tv[1] * e1[2] - tv[2] * e1[1], tv[2] * e1[0] - tv[0] * e1[2], tv[0] * e1[1] - tv[1] * e1[0]};
    const double bv = (u[0] * qv[0] + u[1] * qv[1] + u[2] * qv[2]) * id;
    if (bv < 0.0 || bu + bv > 1.0) continue;
    const double t = (e2[0] * qv[0] + e2[1] * qv[1] + e2[2] * qv[2]) * id;
    if (t > 0.0 && t < best) {
      best = t;
      const double nx = e1[1] * e2[2] - e1[2] * e2[1], ny = e1[2] * e2[0] - e1[0] * e2[2],
                   nz = e1[0] * e2[1] - e1[1] * e2[0];
      const double nn = 1.0 / sqrt(nx * nx + ny * ny + nz * nz);
      n[0] = nx * nn; n[1] = ny * nn; n[2] = nz * nn;
    }
  }
  return best < 1e300 ? best : P.rc;
}

__device__ inline void rot(const double *R, const double *v, double *o) {
  for (int k = 0; k < 3; ++k) o[k] = R[3 * k] * v[0] + R[3 * k + 1] * v[1] + R[3 * k + 2] * v[2];
}
__device__ inline void rot_t(const double *R, const double *v, double *o) {
  for (int k = 0; k < 3; ++k) o[k] = R[k] * v[0] + R[3 + k] * v[1] + R[6 + k] * v[2];
}

// Queue the nodes of A whose ray segment t u (world direction), t in [r_in,
// R_circ], comes within `reach` of the point e (offsets from A's centre);
// returns the count (uniform).  Ends with the queue visible to the wavefront.
__device__ inline int queue_nodes_near(const DevParticle &A, double rin, const double *dirs, const double *e,
                                       double reach, int *queue) {
  const int lane = threadIdx.x;
  const double r2 = reach * reach;
  int nq = 0;
#pragma unroll 1
  for (int m0 = 0; m0 < CONTACT_NODES; m0 += 64) {
    const int m = m0 + lane;
    double w[3];
    rot(A.R, dirs + 3 * m, w);
    const double pr = w[0] * e[0] + w[1] * e[1] + w[2] * e[2];
    const double t = fmin(fmax(pr, rin), A.rc);
    const double dx = t * w[0] - e[0], dy = t * w[1] - e[1], dz = t * w[2] - e[2];
    const bool in = dx * dx + dy * dy + dz * dz < r2;
    const unsigned long long mask = __ballot(in);
    if (in) queue[nq + __popcll(mask & ((1ull << lane) - 1ull))] = m;
    nq += __popcll(mask);
  }
  __syncthreads();
  return nq;
}

// The nodes of A probing the grown B (centre at e from A's centre): adds
// sign * the force and sign * (lever + s) x force to F, T.
// Support function of the body along the unit world direction v: the
// largest (x - X) . v over the body (the circumradius for a mesh).
__device__ inline double support(const DevParticle &P, const double *v) {
  double b[3];
  rot_t(P.R, v, b);
  if (P.shape == 0) return P.prm[0];
  if (P.shape == 1) return (P.prm[0] - P.prm[1]) * (fabs(b[0]) + fabs(b[1]) + fabs(b[2])) + P.prm[1];
  if (P.shape == 2)
    return sqrt(P.prm[0] * P.prm[0] * b[0] * b[0] + P.prm[1] * P.prm[1] * (b[1] * b[1] + b[2] * b[2]));
  return P.rc;
}

template <bool MESH>
__device__ inline void pair_side(const Lattice &L, const DevParticle &A, const DevParticle &B, const double *e,
                                 double zeta, double K, double sign, const double *lever, const double *dirs,
                                 int *queue, double *F, double *T) {
  const int nq = queue_nodes_near(A, inscribed_radius(A), dirs, e, B.rc + zeta, queue);
#pragma unroll 1
  for (int k0 = 0; k0 < nq; k0 += 64) {
    const int k = k0 + (int)threadIdx.x;
    if (k < nq) {
      const double *u = dirs + 3 * queue[k];
      double nb[3];
      const double t = surface_ray<MESH>(L, A, u, nb);
      const double a = (4.0 * M_PI / CONTACT_NODES) * t * t / (u[0] * nb[0] + u[1] * nb[1] + u[2] * nb[2]);
      const double b[3] = {t * u[0], t * u[1], t * u[2]};
      double sv[3], y[3], yb[3];
      rot(A.R, b, sv);
      for (int j = 0; j < 3; ++j) y[j] = sv[j] - e[j];
      rot_t(B.R, y, yb);
      // spheroid: the scaled spheroids s E and E (s^2 the implicit value) are
      // at least (s - 1) min(a, b) apart, a cheap bound before the iteration
      bool far = false;
      if (B.shape == 2) {
        const double kk = yb[0] * yb[0] / (B.prm[0] * B.prm[0]) + (yb[1] * yb[1] + yb[2] * yb[2]) / (B.prm[1] * B.prm[1]);
        far = (sqrt(kk) - 1.0) * fmin(B.prm[0], B.prm[1]) >= zeta;
      }
      // a spheroid's distance and gradient come from one nearest-point iteration
      double gb[3];
      const double d = far ? zeta
                           : (B.shape == 2 ? spheroid_distance_normal(B.prm[0], B.prm[1], yb, gb)
                                           : body_sdf<MESH>(L, B, yb));
      if (d < zeta) {
        double g[3];
        if (B.shape != 2) body_sdf_normal<MESH>(L, B, yb, gb);
        rot(B.R, gb, g);
        const double w = 0.5 * K * a * (zeta - d);
        const double f[3] = {w * g[0], w * g[1], w * g[2]};
        const double r[3] = {lever[0] + sv[0], lever[1] + sv[1], lever[2] + sv[2]};
        for (int j = 0; j < 3; ++j) F[j] += sign * f[j];
        T[0] += sign * (r[1] * f[2] - r[2] * f[1]);
        T[1] += sign * (r[2] * f[0] - r[0] * f[2]);
        T[2] += sign * (r[0] * f[1] - r[1] * f[0]);
      }
    }
  }
  __syncthreads();  // the queue is refilled next
}

// MESH: the particles include mesh shapes (else their code is left out)
template <bool MESH>
__global__ __launch_bounds__(64) void k_contact_shapes(Lattice L, const DevParticle *__restrict__ parts, int n,
                                                       ContactParams c, const double *__restrict__ dirs,
                                                       int *__restrict__ cand, int *__restrict__ ccnt,
                                                       double *__restrict__ out) {
  __shared__ int queue[CONTACT_NODES];
  __shared__ int part[CONTACT_CAND];
  const int pid = blockIdx.x, lane = threadIdx.x;
  const DevParticle &P = parts[pid];
  const int nn[3] = {L.nx, L.ny, L.nz};
  double F[3] = {0.0, 0.0, 0.0}, T[3] = {0.0, 0.0, 0.0};
  const double Rp = cbrt(3.0 * P.V / (4.0 * M_PI));
  // partners in increasing index: the list entries ranked by value
  const int np = min(ccnt[pid], CONTACT_CAND);
  const int mine = lane < np ? cand[(size_t)pid * CONTACT_CAND + lane] : 0;
  __syncthreads();
  if (lane == 0) ccnt[pid] = 0;  // emptied for the next step's k_contact
  if (lane < np) {
    int rank = 0;
    for (int k = 0; k < np; ++k) rank += cand[(size_t)pid * CONTACT_CAND + k] < mine;
    part[rank] = mine;
  }
  __syncthreads();
  for (int k = 0; k < np; ++k) {  // uniform
    const DevParticle &Q = parts[part[k]];
    double e[3], me[3];
    for (int a = 0; a < 3; ++a) {
      double dx = Q.X[a] - P.X[a];
      if (!L.bc[a]) dx = dx > 0.5 * nn[a] ? dx - nn[a] : (dx < -0.5 * nn[a] ? dx + nn[a] : dx);
      e[a] = dx;
      me[a] = -dx;
    }
    // separated along the line of centres by at least the range (support
    // functions): no node of either body comes within the range of the other
    const double dist = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    const double v[3] = {e[0] / dist, e[1] / dist, e[2] / dist}, mv[3] = {-v[0], -v[1], -v[2]};
    if (dist - support(P, v) - support(Q, mv) >= c.range) continue;  // uniform
    const double Rq = cbrt(3.0 * Q.V / (4.0 * M_PI));
    const double K = c.k / (M_PI * (Rp * Rq / (Rp + Rq)) * c.range * c.range);
    const double zero[3] = {0.0, 0.0, 0.0};
    pair_side<MESH>(L, P, Q, e, c.range, K, 1.0, zero, dirs, queue, F, T);
    pair_side<MESH>(L, Q, P, me, c.range, K, -1.0, e, dirs, queue, F, T);
  }
  if (P.shape != 0 && c.kw != 0.0) {
    const double Kw = c.kw / (M_PI * 0.5 * Rp * c.range * c.range);
    const double rin = inscribed_radius(P);
    for (int a = 0; a < 3; ++a) {
      if (!L.bc[a]) continue;
      for (int side = 0; side < 2; ++side) {
        const double hc = side == 0 ? P.X[a] : nn[a] - P.X[a];  // centre distance from the wall
        if (!(hc < P.rc + 0.5 * c.range)) continue;             // uniform
        // nodes whose ray segment reaches closer than zeta/2 to the wall
        int nq = 0;
#pragma unroll 1
        for (int m0 = 0; m0 < CONTACT_NODES; m0 += 64) {
          const int m = m0 + lane;
          double w[3];
          rot(P.R, dirs + 3 * m, w);
          const double wa = side == 0 ? -w[a] : w[a];  // towards the wall
          const bool in = hc - (wa > 0.0 ? P.rc * wa : rin * wa) < 0.5 * c.range;
          const unsigned long long mask = __ballot(in);
          if (in) queue[nq + __popcll(mask & ((1ull << lane) - 1ull))] = m;
          nq += __popcll(mask);
        }
        __syncthreads();
        for (int k0 = 0; k0 < nq; k0 += 64) {
          const int k = k0 + lane;
          if (k < nq) {
            const double *u = dirs + 3 * queue[k];
            double nb[3];
            const double t = surface_ray<MESH>(L, P, u, nb);
            const double wgt = (4.0 * M_PI / CONTACT_NODES) * t * t / (u[0] * nb[0] + u[1] * nb[1] + u[2] * nb[2]);
            const double b[3] = {t * u[0], t * u[1], t * u[2]};
            double sv[3];
            rot(P.R, b, sv);
            const double hs = side == 0 ? P.X[a] + sv[a] : nn[a] - (P.X[a] + sv[a]);
            const double delta = c.range - 2.0 * hs;
            if (delta > 0.0) {
              double f[3] = {0.0, 0.0, 0.0};
              f[a] = (side == 0 ? 1.0 : -1.0) * Kw * wgt * delta;
              F[a] += f[a];
              T[0] += sv[1] * f[2] - sv[2] * f[1];
              T[1] += sv[2] * f[0] - sv[0] * f[2];
              T[2] += sv[0] * f[1] - sv[1] * f[0];
            }
          }
        }
        __syncthreads();
      }
    }
  }
  double v[6] = {F[0], F[1], F[2], T[0], T[1], T[2]};
#pragma unroll
  for (int k = 0; k < 6; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0)
    for (int k = 0; k < 6; ++k) out[(size_t)pid * 6 + k] = v[k];
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

hipError_t launch_mark_learned(DevParticle *parts, int n, const LearnedModes &modes, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mark_learned, dim3(blocks_for(n, 128)), dim3(128), 0, s, parts, n, modes);
  return hipGetLastError();
}

hipError_t launch_fill_int(int *p, int v, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_int, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_bin(const Lattice &L, const DevParticle *parts, int n, int cap, int *tcnt, int *tlist,
                      int *status, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bin, dim3(blocks_for(cap, 64), n), dim3(64), 0, s, L, parts, tcnt, tlist, status);
  return hipGetLastError();
}

hipError_t launch_mea(int prec, const Lattice &L, const void *A, const DevParticle *parts, const int *order, int n,
                      int lmax, int layers, int chunked, double *partial, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 grid(n * ((lmax + layers - 1) / layers));
  HLBM_DISPATCH(prec, {
    if ((unsigned long long)L.N * sizeof(typename ST::S) < (1ull << 32))
      hipLaunchKernelGGL((k_mea<ST, true>), grid, dim3(256), 0, s, L, (const typename ST::S *)A, parts, order, n, lmax, layers, chunked, partial);
    else
      hipLaunchKernelGGL((k_mea<ST, false>), grid, dim3(256), 0, s, L, (const typename ST::S *)A, parts, order, n, lmax, layers, chunked, partial);
  });
  return hipGetLastError();
}

hipError_t launch_contact(const Lattice &L, const DevParticle *parts, int n, const ContactParams &c,
                          const ContactGrid &cg, const ContactWork &w, double *out, int *cand, int *ccnt, int *status,
                          hipStream_t s) {
  if (n <= 0 || !c.on) return hipSuccess;
  if (n < CONTACT_GRID_MIN) {
    const dim3 grid(blocks_for(n, 256), contact_chunks(n));
    hipLaunchKernelGGL(k_contact_pairs, grid, dim3(256), 0, s, L, parts, n, c, out, cand, ccnt, status);
    return hipGetLastError();
  }
  const int ncells = cg.g[0] * cg.g[1] * cg.g[2];
  if (ncells < 1 || ncells > CGRID_MAX) return hipErrorInvalidValue;
  hipError_t e = launch_fill_int(w.gcount, 0, ncells + 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cgrid_count, dim3(blocks_for(n, 256)), dim3(256), 0, s, parts, n, cg, w.gcount, w.gcell,
                     w.gpos);
  hipLaunchKernelGGL(k_cgrid_scan, dim3(1), dim3(1024), 0, s, w.gcount, ncells, w.gfill);
  hipLaunchKernelGGL(k_cgrid_fill, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, w.gcell, w.gfill, w.glist);
  hipLaunchKernelGGL(k_contact, dim3(blocks_for(n, 4)), dim3(256), 0, s, L, n, c, cg, w.gpos, w.gcount, w.gcell,
                     w.glist, out, cand, ccnt, status);
  return hipGetLastError();
}

hipError_t launch_contact_shapes(const Lattice &L, const DevParticle *parts, int n, const ContactParams &c,
                                 const double *dirs, int *cand, int *ccnt, double *out, hipStream_t s) {
  if (n <= 0 || !c.on) return hipSuccess;
  if (L.mesh_nt > 0)
    hipLaunchKernelGGL(k_contact_shapes<true>, dim3(n), dim3(64), 0, s, L, parts, n, c, dirs, cand, ccnt, out);
  else
    hipLaunchKernelGGL(k_contact_shapes<false>, dim3(n), dim3(64), 0, s, L, parts, n, c, dirs, cand, ccnt, out);
  return hipGetLastError();
}

hipError_t launch_eom_bin(const Lattice &L, DevParticle *parts, int n, int lmax, int layers, const double *partial,
                          const ContactParams &c, const double *contact, const double *shapes, int *tcnt, int *tlist,
                          int *status, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (c.on)
    hipLaunchKernelGGL(k_eom_bin<true>, dim3(n), dim3(64), 0, s, L, parts, n, lmax, layers, partial, c, contact,
                       shapes, tcnt, tlist, status);
  else
    hipLaunchKernelGGL(k_eom_bin<false>, dim3(n), dim3(64), 0, s, L, parts, n, lmax, layers, partial, c, contact,
                       shapes, tcnt, tlist, status);
  return hipGetLastError();
}

}  // namespace hlbm
