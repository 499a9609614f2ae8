// hlbm_fields.hip -- gfx950 kernels off the time step: equilibrium
// initialisation of the populations and the observables (moments, u_phys,
// indicator, volume-flux reduction) of the current state.
#include "hlbm_internal.h"
#include "hlbm_tile.h"

namespace hlbm {
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

// Observables of one cell of the current state (Sec. 3.1 moments): rho, the
// bare u, u_phys = u + du/2 with du = B (u_s - u) + (1 - B) a_f from the
// current particles, and B, all in FP64 from the stored populations.
template <class ST, typename G>
__device__ inline void cell_observables(const Lattice &L, const typename ST::S *__restrict__ A,
                                        const CellPos &cp, const PullIdx &P, const TileFields<G> &tf, int nc,
                                        int zz, double &rho, double *u, double *up, double &Bc) {
  using T = typename ST::T;
  T g[Q];
  pull_all<ST>(L, A, cp, P, g);
  G S0 = G(0), S1[3] = {G(0), G(0), G(0)};
  if (nc > 0) {
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
  rho = 1.0 + rho1;
  for (int k = 0; k < 3; ++k) u[k] = j[k] / rho;
  const double s0 = (double)S0;
  Bc = s0 < 1.0 ? s0 : 1.0;
  // the velocity change of the step's coupling per unit density: weight B
  // (exact-difference source) or B_n (partially saturated collision)
  const double Bw = L.psm ? Bc * L.tau_mh / ((1.0 - Bc) + L.tau_mh) : Bc;
  for (int k = 0; k < 3; ++k) {
    const double us = s0 > 0.0 ? (double)S1[k] / s0 : 0.0;
    const double du = Bw * (us - u[k]) + (1.0 - Bw) * L.af[k];
    up[k] = u[k] + 0.5 * du;
  }
}

// Observables written as planes of OutT (FP64 or FP32, rounded to nearest),
// in the order rho, u, u_phys, B (only the selected ones).
template <class ST, typename OutT>
__global__ __launch_bounds__(256) void k_fields(Lattice L, const typename ST::S *__restrict__ A,
                                                const DevParticle *__restrict__ parts,
                                                const int *__restrict__ tcnt,
                                                const int *__restrict__ tlist, unsigned mask,
                                                OutT *__restrict__ out) {
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
    const PullIdx P = pull_index(L, cp);
    const long long cell = P.cell;
    double rho, u[3], up[3], Bc;
    cell_observables<ST, G>(L, A, cp, P, tf, tc.n, zz, rho, u, up, Bc);
    long long plane = 0;
    if (mask & 1u) { out[plane * L.N + cell] = (OutT)rho; plane += 1; }
    if (mask & 2u) { for (int k = 0; k < 3; ++k) out[(plane + k) * L.N + cell] = (OutT)u[k]; plane += 3; }
    if (mask & 4u) { for (int k = 0; k < 3; ++k) out[(plane + k) * L.N + cell] = (OutT)up[k]; plane += 3; }
    if (mask & 8u) { out[plane * L.N + cell] = (OutT)Bc; }
  }
}

// Volume-flux reduction, pass 1: per tile, in FP64, the sums of u_phys over
// all cells, of u_phys over the pure-fluid cells (B = 0) and the number of
// those cells -> partial[tile][7].  Lanes sum their column over the tile's
// z-layers, then a fixed wavefront butterfly and the four wavefronts in order.
template <class ST>
__global__ __launch_bounds__(256) void k_mean_velocity_tiles(Lattice L, const typename ST::S *__restrict__ A,
                                                             const DevParticle *__restrict__ parts,
                                                             const int *__restrict__ tcnt,
                                                             const int *__restrict__ tlist,
                                                             double *__restrict__ partial) {
  using G = typename ST::G;
  __shared__ TileCands<G> tc;
  __shared__ TileFields<G> tf;
  __shared__ double red[4][7];
  const int tile = xcd_chunk(blockIdx.x, L.ntiles);
  const int tx = tile % L.ntx;
  const int ty = (tile / L.ntx) % L.nty;
  const int tz = tile / (L.ntx * L.nty);
  load_candidates<G>(L, parts, tcnt, tlist, tile, tc);
  tile_coupling<G>(L, tc, tx, ty, tz, tf);
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int zz = 0; zz < TZ; ++zz) {
    CellPos cp;
    cp.x = tx * TX + lane_id();
    cp.y = ty * TY + wave_id();
    cp.z = tz * TZ + zz;
    if (cp.z >= L.nz || cp.y >= L.ny) break;
    cp.act = cp.x < L.nx;
    if (!cp.act) continue;
    const PullIdx P = pull_index(L, cp);
    double rho, u[3], up[3], Bc;
    cell_observables<ST, G>(L, A, cp, P, tf, tc.n, zz, rho, u, up, Bc);
    for (int k = 0; k < 3; ++k) acc[k] += up[k];
    if (Bc == 0.0) {
      for (int k = 0; k < 3; ++k) acc[3 + k] += up[k];
      acc[6] += 1.0;
    }
  }
#pragma unroll
  for (int k = 0; k < 7; ++k) acc[k] = wave_sum(acc[k]);
  if (lane_id() == 0)
    for (int k = 0; k < 7; ++k) red[wave_id()][k] = acc[k];
  __syncthreads();
  if (threadIdx.x < 7) {
    const int k = threadIdx.x;
    partial[(size_t)tile * 7 + k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
  }
}

// Pass 2: one workgroup sums the tile records in a fixed order (thread t takes
// tiles t, t + 256, ..., then the fixed butterfly and the wavefronts in order).
__global__ __launch_bounds__(256) void k_mean_velocity_sum(const double *__restrict__ partial, int ntiles,
                                                           double *__restrict__ out) {
  __shared__ double red[4][7];
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int t = threadIdx.x; t < ntiles; t += 256)
    for (int k = 0; k < 7; ++k) acc[k] += partial[(size_t)t * 7 + k];
#pragma unroll
  for (int k = 0; k < 7; ++k) acc[k] = wave_sum(acc[k]);
  if (lane_id() == 0)
    for (int k = 0; k < 7; ++k) red[wave_id()][k] = acc[k];
  __syncthreads();
  if (threadIdx.x < 7) {
    const int k = threadIdx.x;
    out[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
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

hipError_t launch_set_fields(int prec, const Lattice &L, void *A, const double *rho, const double *u,
                             hipStream_t s) {
  HLBM_DISPATCH(prec, hipLaunchKernelGGL(k_set_fields<ST>, dim3(blocks_for(L.N, 256)), dim3(256), 0, s,
                                         L, (typename ST::S *)A, rho, u));
  return hipGetLastError();
}

hipError_t launch_fields(int prec, const Lattice &L, const void *A, const DevParticle *parts,
                         const int *tcnt, const int *tlist, unsigned mask, int out_f32, void *out,
                         hipStream_t s) {
  if (out_f32) {
    HLBM_DISPATCH(prec, hipLaunchKernelGGL((k_fields<ST, float>), dim3(L.ntiles), dim3(256), 0, s, L,
                                           (const typename ST::S *)A, parts, tcnt, tlist, mask, (float *)out));
  } else {
    HLBM_DISPATCH(prec, hipLaunchKernelGGL((k_fields<ST, double>), dim3(L.ntiles), dim3(256), 0, s, L,
                                           (const typename ST::S *)A, parts, tcnt, tlist, mask, (double *)out));
  }
  return hipGetLastError();
}

hipError_t launch_mean_velocity(int prec, const Lattice &L, const void *A, const DevParticle *parts,
                                const int *tcnt, const int *tlist, double *partial, double *out,
                                hipStream_t s) {
  HLBM_DISPATCH(prec, hipLaunchKernelGGL(k_mean_velocity_tiles<ST>, dim3(L.ntiles), dim3(256), 0, s, L,
                                         (const typename ST::S *)A, parts, tcnt, tlist, partial));
  hipLaunchKernelGGL(k_mean_velocity_sum, dim3(1), dim3(256), 0, s, (const double *)partial, L.ntiles, out);
  return hipGetLastError();
}

}  // namespace hlbm
