// hlbm_lattice.hip -- the gfx950 collide-and-stream kernel of the HLBM time
// step.
//
//   k_collide   one workgroup per tile of 64 x 4 x 4 cells: the tile's
//               particles staged in LDS, the indicator and solid velocity of
//               the tile's cells accumulated in LDS by a dense pre-pass over
//               each particle's part of the tile, then per cell: pull,
//               moments, exact-difference source (or the partially
//               saturated collision), BGK, store.
#include "hlbm_internal.h"
#include "hlbm_tile.h"

namespace hlbm {

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

// At least 5 wavefronts per SIMD asked of the register allocator: the FP32
// and FP16S instances then fit in 76 VGPRs (6 waves) and the partially
// saturated ones in 96 (5 waves), which the memory-bound loop turns into
// time (mixed256 FP16S 342 -> 321 us, hindered384 PSM 1883 -> 1778 us).
template <class ST, bool PSM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_collide(Lattice L, const typename ST::S *__restrict__ A,
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
    // one flag per wavefront, raised by its first unstable lane
    const unsigned long long bad = __ballot(cp.act && !(rho > (T)0 && usq < (T)0.09));
    if (bad && lane_id() == __ffsll((long long)bad) - 1) atomicOr(status, ST_UNSTABLE);
    const T Kr1 = K * rho1, Krho = K * rho;
    const T o3 = (T)3 * Krho, e45 = (T)4.5 * Krho;  // e_i = base + e45 (c.u)^2 + o3 c.u
    const T base = Kr1 - (T)1.5 * Krho * usq;
    T out[Q];
    bool psm_cell = false;
    if constexpr (PSM) psm_cell = S0 > G(0);
    if (psm_cell) {
      // partially saturated collision (Noble and Torczynski 1998): with the
      // solid weight B_n = B (tau - 1/2) / ((1 - B) + (tau - 1/2)) and the
      // non-equilibrium parts n_i = s_i - e_i(u),
      //   s*_i = s_i - (1 - B_n) n_i / tau + B_n (n_opp(i) + e_i(u_s) - s_i)
      //          + (1 - B_n) (e_i(u + a_f) - e_i(u))
      const T Bt = (T)(S0 < G(1) ? S0 : G(1));
      const G is0 = frcp(S0);
      const T usx = (T)(S1[0] * is0), usy = (T)(S1[1] * is0), usz = (T)(S1[2] * is0);
      const T tm = (T)L.tau_mh;
      const T Bn = Bt * tm / (((T)1 - Bt) + tm);
      const T keep = omega * ((T)1 - Bn), fa = (T)1 - Bn;
      const T sbase = Kr1 - (T)1.5 * Krho * (usx * usx + usy * usy + usz * usz);
      const T vx = ux + afx, vy = uy + afy, vz = uz + afz;
      const T dE0 = (T)-1.5 * Krho * ((vx * vx + vy * vy + vz * vz) - usq);
      const T n0 = s[0] - base;
      out[0] = s[0] - keep * n0 + Bn * (sbase - base) + fa * dE0;
#pragma unroll
      for (int i = 1; i < Q; i += 2) {
        const T cu = (T)kCX[i] * ux + (T)kCY[i] * uy + (T)kCZ[i] * uz;
        const T E = base + e45 * cu * cu, O = o3 * cu;
        const T ni = s[i] - (E + O), no = s[i + 1] - (E - O);
        const T cs = (T)kCX[i] * usx + (T)kCY[i] * usy + (T)kCZ[i] * usz;
        const T sE = sbase + e45 * cs * cs, sO = o3 * cs;
        const T cd = (T)kCX[i] * afx + (T)kCY[i] * afy + (T)kCZ[i] * afz;
        const T dE = dE0 + e45 * cd * (cd + (T)2 * cu), dO = o3 * cd;
        out[i] = s[i] - keep * ni + Bn * (no + (sE + sO) - s[i]) + fa * (dE + dO);
        out[i + 1] = s[i + 1] - keep * no + Bn * (ni + (sE - sO) - s[i + 1]) + fa * (dE - dO);
      }
    } else {
    // plain BGK, then the exact-difference source e_i(u + du) - e_i(u) where
    // the cell is coupled
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
  if (L.psm) {
    HLBM_DISPATCH(prec, hipLaunchKernelGGL((k_collide<ST, true>), dim3(L.ntiles), dim3(256), 0, s, L,
                                           (const typename ST::S *)A, (typename ST::S *)B, parts, tcnt, tlist,
                                           tcnt_clear, status));
  } else {
    HLBM_DISPATCH(prec, hipLaunchKernelGGL((k_collide<ST, false>), dim3(L.ntiles), dim3(256), 0, s, L,
                                           (const typename ST::S *)A, (typename ST::S *)B, parts, tcnt, tlist,
                                           tcnt_clear, status));
  }
  return hipGetLastError();
}

}  // namespace hlbm
